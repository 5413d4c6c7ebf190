"""Free-energy estimators of the parallel pulling protocol -- TEST INFRASTRUCTURE ONLY.

Everything is computed in fp64 from the pooled xi samples of each window, by
the definitions in the paper (arXiv:1105.4840):

* step-wise work of the i-th step, the summand of Eq. 9:
  dW_i(x) = k/2 [(x - lambda_{i+1})^2 - (x - lambda_i)^2];
* JE along the windows, Eq. 12.  The windows are independent (Sec. II, the
  remark that rho(W_mech) is proportional to the product of the rho(x_i)), so
  <exp(-beta W_mech)> factorises into per-window averages and
  dF^JE(lambda_j) = sum_{i<j} -kT ln < exp(-beta dW_i) >_i;
* the alternative formula Eq. 14 and the Gaussian formula Eq. 13 (App. B.5),
  read with the actual per-step increment dlambda_i = lambda_{i+1} - lambda_i;
* the combined estimate (dF^JE + dF_fluct)/2 with uncertainty
  (dF^JE - dF_fluct)/2 (Sec. IV B and IV D);
* gamma_i^2 = k sigma_i^2 / kT (Sec. II, below Eq. 12);
* jackknife standard errors over replica blocks, the JE variance formula of
  Sec. IV A / App. C, Kish effective sample size and adjacent-window overlap;
* with the unrestrained ensemble x_0 sampled as well (Sec. II): the turn-on
  free energy dF(lambda, k) = F(lambda, k) - F_0 by Eq. 5 (restrained window)
  and by Eq. 6 (x_0), the bounds of Eq. 7, the average of Eq. 10 over the
  independent ensembles x_0, x_1 .. x_s, and G of Eq. 15.
"""
import numpy as np

from . import appc


def logsumexp(a):
    """ln sum exp(a), by its definition with the maximum factored out."""
    a = np.asarray(a, dtype=np.float64)
    if a.size == 0:
        return -np.inf
    m = np.max(a)
    return m + np.log(np.sum(np.exp(a - m)))


def step_work(x, lam_i, lam_next, k):
    """Work of moving the restraint centre from lam_i to lam_next at fixed x (Eq. 9 summand)."""
    return 0.5 * k * ((x - lam_next) ** 2 - (x - lam_i) ** 2)


def block_of(replica, n_replicas, n_blocks):
    """Jackknife block of a replica: contiguous blocks, block = floor(r B / R)."""
    return (replica * n_blocks) // n_replicas


def pooled(xi, kept, window, n_replicas, replicas=None):
    """All kept samples of one window in replica order."""
    rows = range(n_replicas) if replicas is None else replicas
    base = window * n_replicas
    parts = [xi[base + r, :kept[base + r]] for r in rows]
    return np.concatenate(parts) if parts else np.zeros(0)


def window_stats(samples, w, lam, k, kT):
    """Per-window statistics used by the estimators."""
    s = len(lam)
    beta = 1.0 / kT
    n = samples.size
    out = {"n": n}
    out["mean"] = np.mean(samples) if n else np.nan
    out["var"] = np.var(samples, ddof=1) if n > 1 else np.nan
    if w + 1 < s:
        a = -beta * step_work(samples, lam[w], lam[w + 1], k)
        out["lse_fwd"] = logsumexp(a)
        out["lse_fwd2"] = logsumexp(2.0 * a)
    else:
        out["lse_fwd"] = out["lse_fwd2"] = np.nan
    if w > 0:
        ar = -beta * step_work(samples, lam[w], lam[w - 1], k)
        out["lse_rev"] = logsumexp(ar)
        out["lse_rev2"] = logsumexp(2.0 * ar)
    else:
        out["lse_rev"] = out["lse_rev2"] = np.nan
    out["min"] = np.min(samples) if n else np.nan
    out["max"] = np.max(samples) if n else np.nan
    return out


def profiles(stats, lam, k, kT):
    """dF^JE, dF_fluct, dF^G, dF_com, unc and the reverse-direction JE profile."""
    s = len(lam)
    je = np.zeros(s); fl = np.zeros(s); g = np.zeros(s); rev = np.zeros(s)
    for j in range(1, s):
        i = j - 1
        dl = lam[i + 1] - lam[i]
        st = stats[i]
        # Eq. 12 factorised over independent windows
        je[j] = je[j - 1] - kT * (st["lse_fwd"] - np.log(st["n"]))
        # Eq. 14 with the actual increment
        fl[j] = fl[j - 1] + k * dl * (lam[i] - st["mean"])
        # Eq. 13 / App. B.5 with the actual increment
        gamma2 = k * st["var"] / kT
        g[j] = g[j - 1] + k * dl * (lam[i] - st["mean"]) + 0.5 * k * dl * dl * (1.0 - gamma2)
        # reverse perturbation from window i+1 to window i
        sj = stats[j]
        rev[j] = rev[j - 1] + kT * (sj["lse_rev"] - np.log(sj["n"]))
    com = 0.5 * (je + fl)
    unc = 0.5 * (je - fl)
    # Eqs. 14 and 13 as printed, with lambda_j as the end point: the increment
    # (lambda_j - lambda_1)/j in place of each step (j counted from 1)
    fl_lit = np.zeros(s); g_lit = np.zeros(s)
    for j in range(1, s):
        n_pts = j + 1
        span = lam[j] - lam[0]
        s1 = sum(lam[i] - stats[i]["mean"] for i in range(j))
        s2 = sum(1.0 - k * stats[i]["var"] / kT for i in range(j))
        fl_lit[j] = k * span * s1 / n_pts
        g_lit[j] = k * span ** 2 / (2.0 * n_pts) * s2 / n_pts + fl_lit[j]
    return {"dF_je": je, "dF_fluct": fl, "dF_gauss": g, "dF_com": com, "dF_unc": unc, "dF_rev": rev,
            "dF_fluct_literal": fl_lit, "dF_gauss_literal": g_lit}


def gauss_fit(counts, n, x_min, dx, mean, sd):
    """The paper's sigma (Sec. IV A: sigma_i by least-squares fitting of the x_i
    distribution): the Gaussian A exp(-(x - mu)^2 / (2 sigma^2)) fitted in least
    squares to the histogram density counts / (n dx) at the bin centres.  The
    paper names no algorithm; the one taken here is Levenberg-Marquardt from the
    sample moments with a fixed schedule, so that a histogram whose least-squares
    problem has several minima (one that shows only part of the distribution)
    still gets one defined answer:
      start A = 1 / (sd sqrt(2 pi)), mu = mean, sigma = sd, damping l = 1e-3;
      step: solve (J^T J + l diag(J^T J)) d = J^T r for the residual r = y - f;
      accept if the squared residual does not grow (then l = max(l/10, 1e-15)),
      else l = 10 l; stop once every component of d is within 1e-14 of its
      parameter's scale (mu's: |mu| + sigma), when l exceeds 1e12, or after 200
      steps.  Returns (A, mu, sigma), or NaNs for fewer than 3 samples or fewer
    than 3 non-empty bins."""
    counts = np.asarray(counts, dtype=np.float64)
    if not (n > 2) or not (sd > 0) or np.count_nonzero(counts) < 3:   # three parameters need three points
        return np.nan, np.nan, np.nan
    x = x_min + (np.arange(len(counts)) + 0.5) * dx
    y = counts / (n * dx)

    def cost(A, mu, sg):
        return float(np.sum((y - A * np.exp(-(x - mu) ** 2 / (2.0 * sg * sg))) ** 2))
    A, mu, sg = 1.0 / (sd * np.sqrt(2.0 * np.pi)), float(mean), float(sd)
    lm = 1e-3
    c0 = cost(A, mu, sg)
    for _ in range(200):
        d = x - mu
        e = np.exp(-d * d / (2.0 * sg * sg))
        f = A * e
        r = y - f
        J = np.stack([e, f * d / sg ** 2, f * d * d / sg ** 3], axis=1)
        JtJ = J.T @ J
        Jtr = J.T @ r
        M = JtJ + lm * np.diag(np.diag(JtJ))
        with np.errstate(all="ignore"):
            step = np.linalg.solve(M, Jtr) if np.linalg.det(M) != 0 else np.full(3, np.nan)
        done = (abs(step[0]) <= 1e-14 * abs(A) and abs(step[1]) <= 1e-14 * (abs(mu) + sg)
                and abs(step[2]) <= 1e-14 * sg)
        nA, nm, ns = A + step[0], mu + step[1], abs(sg + step[2])
        with np.errstate(all="ignore"):
            c1 = cost(nA, nm, ns)
        if c1 <= c0:
            A, mu, sg, c0 = nA, nm, ns, c1
            lm = max(lm * 0.1, 1e-15)
        else:
            lm *= 10.0
        if done or lm > 1e12:
            break
    return A, mu, sg


def turn_on_values(x1, xs, x0, lam, k, kT, je_s):
    """Turn-on estimates from the samples of window 1 (x1), window s (xs) and the
    unrestrained ensemble (x0); je_s = dF^JE(lambda_s) of the same samples."""
    beta = 1.0 / kT
    l1, ls = lam[0], lam[-1]
    out = {}
    # Eq. 5: exp(beta dF) = < exp(+beta k/2 (x - lambda)^2) > in the restrained ensemble
    out["eq5_first"] = kT * (logsumexp(0.5 * beta * k * (x1 - l1) ** 2) - np.log(x1.size))
    out["eq5_last"] = kT * (logsumexp(0.5 * beta * k * (xs - ls) ** 2) - np.log(xs.size))
    # Eq. 6: exp(-beta dF) = < exp(-beta k/2 (x_0 - lambda)^2) > in the unrestrained ensemble
    out["eq6_first"] = -kT * (logsumexp(-0.5 * beta * k * (x0 - l1) ** 2) - np.log(x0.size))
    out["eq6_last"] = -kT * (logsumexp(-0.5 * beta * k * (x0 - ls) ** 2) - np.log(x0.size))
    # Eq. 10: W_total = k/2 (x_0 - lambda_1)^2 + W_mech - k/2 (x_s - lambda_s)^2 with every
    # x_i from its own ensemble, so the average factorises
    out["eq10_log"] = -beta * (out["eq6_first"] + je_s - out["eq5_last"])
    return out


def turn_on(prob, xi, kept, je):
    """Turn-on outputs (Eqs. 5-7, 10) with jackknife errors, and G of Eq. 15 with its
    error; je is the dF^JE profile of the same samples."""
    lam = np.asarray(prob["lambda"], dtype=np.float64)
    k = float(prob["k"]); kT = float(prob["kT"])
    s = len(lam)
    R = int(prob["n_replicas"])
    B = max(1, min(int(prob.get("n_blocks", 32)), R))
    x1, xs, x0 = (pooled(xi, kept, w, R) for w in (0, s - 1, s))
    res = turn_on_values(x1, xs, x0, lam, k, kT, je[-1])
    # Eq. 15: G(lambda_j, lambda_1) = dF^JE(lambda_j) - dF(lambda_1, k), dF by Eq. 5
    G = je - res["eq5_first"]
    # Eq. 7: <k/2 (x_1 - lambda)^2>_lambda <= dF(lambda, k) <= <k/2 (x_0 - lambda)^2>_0
    res["lower_first"] = 0.5 * k * np.mean((x1 - lam[0]) ** 2)
    res["upper_first"] = 0.5 * k * np.mean((x0 - lam[0]) ** 2)
    res["lower_last"] = 0.5 * k * np.mean((xs - lam[-1]) ** 2)
    res["upper_last"] = 0.5 * k * np.mean((x0 - lam[-1]) ** 2)
    res["free_n"] = x0.size
    res["free_mean"] = np.mean(x0)
    res["free_std"] = np.std(x0, ddof=1)
    keys = ("eq5_first", "eq6_first", "eq5_last", "eq6_last", "eq10_log")
    if B > 1:
        blocks = block_of(np.arange(R), R, B)
        loo = {key: [] for key in keys + ("G",)}
        for b in range(B):
            keep_reps = np.nonzero(blocks != b)[0]
            st_b = [window_stats(pooled(xi, kept, w, R, keep_reps), w, lam, k, kT) for w in range(s)]
            je_b = profiles(st_b, lam, k, kT)["dF_je"]
            xb = [pooled(xi, kept, w, R, keep_reps) for w in (0, s - 1, s)]
            v = turn_on_values(*xb, lam, k, kT, je_b[-1])
            v["G"] = je_b - v["eq5_first"]
            for key in loo:
                loo[key].append(v[key])
        se = {}
        for key in loo:
            th = np.array(loo[key])
            se[key] = np.sqrt((B - 1) / B * np.sum((th - th.mean(axis=0)) ** 2, axis=0))
        for key in keys:
            res[key + "_se"] = float(se[key])
        G_se = se["G"]
    else:
        for key in keys:
            res[key + "_se"] = np.nan
        G_se = np.full(s, np.nan)
    return res, G, G_se


def histograms(xi, kept, prob):
    """Counts of xi in K bins of width dxi from xi_min; bin b = floor((xi - xi_min)/dxi)."""
    lam = np.asarray(prob["lambda"], dtype=np.float64)
    R = int(prob["n_replicas"])
    K = int(prob["xi_nbins"])
    x0 = float(prob["xi_min"]); dx = float(prob["xi_bin"])
    hist = np.zeros((len(lam), K), dtype=np.int64)
    uo = np.zeros((len(lam), 2), dtype=np.int64)
    for w in range(len(lam)):
        smp = pooled(xi, kept, w, R)
        b = np.floor((smp - x0) / dx).astype(np.int64)
        uo[w, 0] = np.count_nonzero(b < 0)
        uo[w, 1] = np.count_nonzero(b >= K)
        inr = b[(b >= 0) & (b < K)]
        hist[w] = np.bincount(inr, minlength=K)
    return hist, uo


def estimate(prob, xi, kept, with_appc=True):
    """All outputs of one protocol run, from the oracle's sample streams."""
    lam = np.asarray(prob["lambda"], dtype=np.float64)
    k = float(prob["k"]); kT = float(prob["kT"])
    s = len(lam)
    R = int(prob["n_replicas"])
    B = int(prob.get("n_blocks", 32))
    B = max(1, min(B, R))

    stats = [window_stats(pooled(xi, kept, w, R), w, lam, k, kT) for w in range(s)]
    res = profiles(stats, lam, k, kT)

    # jackknife over replica blocks (block b removed from every window)
    blocks = [block_of(np.arange(R), R, B) == b for b in range(B)]
    loo = {key: [] for key in ("dF_je", "dF_fluct", "dF_gauss", "dF_com")}
    if B > 1:
        for b in range(B):
            keep_reps = np.nonzero(~blocks[b])[0]
            st_b = [window_stats(pooled(xi, kept, w, R, keep_reps), w, lam, k, kT) for w in range(s)]
            pr = profiles(st_b, lam, k, kT)
            for key in loo:
                loo[key].append(pr[key])
        for key in loo:
            th = np.array(loo[key])
            res[key + "_se"] = np.sqrt((B - 1) / B * np.sum((th - th.mean(axis=0)) ** 2, axis=0))
    else:
        for key in loo:
            res[key + "_se"] = np.full(s, np.nan)

    n = np.array([st["n"] for st in stats], dtype=np.int64)
    mean = np.array([st["mean"] for st in stats])
    var = np.array([st["var"] for st in stats])
    res["n_samples"] = n
    res["xi_mean"] = mean
    res["xi_std"] = np.sqrt(var)
    res["gamma2"] = k * var / kT
    res["lse_fwd"] = np.array([st["lse_fwd"] for st in stats])
    res["lse_rev"] = np.array([st["lse_rev"] for st in stats])
    res["xi_min_sample"] = np.array([st["min"] for st in stats])
    res["xi_max_sample"] = np.array([st["max"] for st in stats])
    # Kish effective sample fraction of the exponential weights, per forward step
    res["kish_frac"] = np.array([np.exp(2 * st["lse_fwd"] - st["lse_fwd2"]) / st["n"]
                                 if i + 1 < s else np.nan for i, st in enumerate(stats)])
    res["n_blown_up"] = np.array([int(np.count_nonzero(
        kept[w * R:(w + 1) * R] < (xi.shape[1] if xi.ndim == 2 else 0))) for w in range(s)])

    hist, uo = histograms(xi, kept, prob)
    res["xi_hist"] = hist
    res["xi_under_over"] = uo

    # overlap diagnostics for each adjacent pair (Sec. III, Sec. IV B, Sec. V)
    dl = np.diff(lam)
    sig = np.sqrt(var)
    res["dlambda_over_sigma"] = np.abs(dl) / sig[:-1]
    # distance from the centre of the distribution to its end in the pulling direction
    reach = np.where(dl > 0, res["xi_max_sample"][:-1] - mean[:-1], mean[:-1] - res["xi_min_sample"][:-1])
    res["reach"] = reach
    res["dlambda_over_reach"] = np.abs(dl) / reach
    res["criterion_ok"] = np.abs(dl) <= reach
    rho = hist / np.maximum(n[:, None], 1)
    res["overlap_ovl"] = np.sum(np.minimum(rho[:-1], rho[1:]), axis=1)

    # sigma_i by least-squares fitting (Sec. IV A), gamma_i^2 from it, and Eq. 13 with it
    sig_lsq = np.array([gauss_fit(hist[w], n[w], float(prob["xi_min"]), float(prob["xi_bin"]), mean[w],
                                  np.sqrt(var[w]) if n[w] > 1 else np.nan)[2] for w in range(s)])
    res["sigma_lsq"] = sig_lsq
    res["gamma2_lsq"] = k * sig_lsq ** 2 / kT
    g = np.zeros(s)
    for j in range(1, s):
        i = j - 1
        dl = lam[i + 1] - lam[i]
        g[j] = g[j - 1] + k * dl * (lam[i] - mean[i]) + 0.5 * k * dl * dl * (1.0 - res["gamma2_lsq"][i])
    res["dF_gauss_lsq"] = g

    if with_appc and int(prob.get("w_half_bins", 0)) > 0:
        res.update(appc.work_distributions(prob, hist, n))
        res.update(appc.work_distributions_literal(prob, hist, n))
        res.update(appc.work_distributions_reverse(prob, hist, n, res["work_hist"]))
    if prob.get("free_ensemble", False):
        on, res["G"], res["G_se"] = turn_on(prob, xi, kept, res["dF_je"])
        res["turn_on"] = on
        x0 = pooled(xi, kept, s, R)
        b0 = np.floor((x0 - float(prob["xi_min"])) / float(prob["xi_bin"])).astype(np.int64)
        K = int(prob["xi_nbins"])
        res["xi_hist_free"] = np.bincount(b0[(b0 >= 0) & (b0 < K)], minlength=K)
        on["free_under"] = int(np.count_nonzero(b0 < 0))
        on["free_over"] = int(np.count_nonzero(b0 >= K))
        on["free_blown"] = int(np.count_nonzero(kept[s * R:(s + 1) * R] < (xi.shape[1] if xi.ndim == 2 else 0)))
    return res
