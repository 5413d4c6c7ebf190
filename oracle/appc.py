"""Work distributions from reaction-coordinate distributions (App. C) -- TEST INFRASTRUCTURE ONLY.

The paper builds the distribution Omega_j of the mechanical work W_mech needed
to reach lambda_j by repeatedly folding in the distribution rho_{j-1} of x at
the previous window: a work bin w of Omega_{j-1} combined with an x bin b of
rho_{j-1} lands in bin floor(W/dW) with W = w dW + dW_{j-1}(x_b), and carries
probability rho_{j-1}(b) Omega_{j-1}(w).

Readings taken here where the appendix leaves a choice:

* the per-step increment is dlambda_i = lambda_{i+1} - lambda_i (not
  (lambda_s - lambda_1)/s);
* contributions are accumulated (+=) into a work bin, also for the first
  step, since several x bins can land in one work bin;
* floor is the mathematical floor; since w is an integer,
  floor(w + dW/dW_bin) = w + floor(dW/dW_bin), so each x bin contributes an
  integer shift s_b = floor(dW_{j-1}(x_b) / dW_bin) that is computed once;
* the x representative of bin b is its centre xi_min + (b + 1/2) dxi;
* the recursion runs to j = s, so the last window of the profile has a
  distribution too; Omega_1 is the point mass at W = 0 (no step taken);
* work outside [-M dW, (M+1) dW) is dropped and reported as lost mass.

The reverse path (lambda_j back to lambda_1) is built the same way from the
windows the reverse steps start from, and checked against the forward one
with Crooks' fluctuation theorem and the overlap of the two (Sec. V).

From Omega_j: dF^JE by Eq. 12 / App. B.5 (normalised average of
exp(-beta W)), with W taken at the left bin edge w dW (each of the j-1 floors
rounds down, so the true work lies in [w dW, (w + j - 1) dW)), and with the
mid-point w dW + (j-1) dW/2; and the variance formula of Sec. IV A / App. C,
sigma_W^2/Q + beta^2 sigma_W^4 / (2 (Q - 1)) with Q the number of non-zero bins.
"""
import numpy as np


def paper_variance(sigma_w, Q, kT):
    """Variance of dF^JE, sigma_W^2/Q + beta^2 sigma_W^4 / (2 (Q-1))."""
    beta = 1.0 / kT
    if Q <= 1:
        return 0.0
    return sigma_w ** 2 / Q + beta ** 2 * sigma_w ** 4 / (2.0 * (Q - 1))


def bin_shifts(prob, window):
    """Integer work-bin shift of every x bin for the step window -> window + 1."""
    lam = np.asarray(prob["lambda"], dtype=np.float64)
    k = float(prob["k"])
    K = int(prob["xi_nbins"])
    x0 = float(prob["xi_min"]); dx = float(prob["xi_bin"]); dWb = float(prob["w_bin"])
    xb = x0 + (np.arange(K) + 0.5) * dx
    dW = 0.5 * k * ((xb - lam[window + 1]) ** 2 - (xb - lam[window]) ** 2)
    return np.floor(dW / dWb).astype(np.int64)


def work_distributions(prob, hist, n):
    """Omega_j for j = 1..s and the quantities derived from them."""
    lam = np.asarray(prob["lambda"], dtype=np.float64)
    s = len(lam)
    kT = float(prob["kT"]); beta = 1.0 / kT
    M = int(prob["w_half_bins"]); dWb = float(prob["w_bin"])
    nb = 2 * M + 1
    omega = np.zeros((s, nb))
    omega[0, M] = 1.0                                  # W = 0 before any step
    lost = np.zeros(s)
    for j in range(1, s):
        rho = hist[j - 1] / max(int(n[j - 1]), 1)        # probability per x bin
        shifts = bin_shifts(prob, j - 1)
        prev = omega[j - 1]
        cur = omega[j]
        for b in np.nonzero(rho)[0]:                   # the paper's loop over x bins
            sb = int(shifts[b])
            # every work bin w1 of Omega_{j-1} moves to w1 + sb (index space: +M offset)
            lo = max(0, -sb); hi = min(nb, nb - sb)
            if lo < hi:
                cur[lo + sb:hi + sb] += rho[b] * prev[lo:hi]
        lost[j] = 1.0 - cur.sum()
    w = np.arange(-M, M + 1, dtype=np.float64)
    je_left = np.full(s, np.nan); je_mid = np.full(s, np.nan)
    var_paper = np.zeros(s); sigma_w = np.zeros(s); q_bins = np.zeros(s, dtype=np.int64)
    for j in range(s):
        om = omega[j]
        tot = om.sum()
        if tot <= 0:
            continue
        W_left = w * dWb
        W_mid = W_left + 0.5 * j * dWb
        # normalised exponential average (App. B.5)
        je_left[j] = -kT * np.log(np.sum(om * np.exp(-beta * W_left)) / tot)
        je_mid[j] = -kT * np.log(np.sum(om * np.exp(-beta * W_mid)) / tot)
        mean_w = np.sum(om * W_left) / tot
        sigma_w[j] = np.sqrt(max(np.sum(om * (W_left - mean_w) ** 2) / tot, 0.0))
        q_bins[j] = np.count_nonzero(om)
        var_paper[j] = paper_variance(sigma_w[j], q_bins[j], kT) if j > 0 else 0.0
    return {"work_hist": omega, "work_lost": lost, "dF_je_hist": je_left, "dF_je_hist_mid": je_mid,
            "sigma_w": sigma_w, "q_bins": q_bins, "dF_je_var_paper": var_paper}


def work_distributions_literal(prob, hist, n):
    """App. C as printed: the x representative of bin b is x = (b+1) dxi past
    xi_min (x = j dx with j counted from 1), the work W = w dW + dW_{j-1}(x) of
    a pair goes to bin [W / dW] taken as C's conversion to an integer
    (truncation toward zero), and each Omega_j (j >= 2) has its bin at W = 0
    replaced by the mean of its two neighbours, the smoothing the paper applies
    to the spike that this rounding makes there.  Contributions are
    accumulated (+=).  Returns the Omega_j and dF^JE from their normalised
    exponential averages with W at w dW."""
    lam = np.asarray(prob["lambda"], dtype=np.float64)
    s = len(lam)
    k = float(prob["k"]); kT = float(prob["kT"]); beta = 1.0 / kT
    M = int(prob["w_half_bins"]); dWb = float(prob["w_bin"])
    K = int(prob["xi_nbins"]); x0 = float(prob["xi_min"]); dx = float(prob["xi_bin"])
    nb = 2 * M + 1
    wv = np.arange(-M, M + 1, dtype=np.float64)
    omega = np.zeros((s, nb))
    omega[0, M] = 1.0
    xb = x0 + (np.arange(K) + 1.0) * dx
    for j in range(1, s):
        rho = hist[j - 1] / max(int(n[j - 1]), 1)
        f = 0.5 * k * ((xb - lam[j]) ** 2 - (xb - lam[j - 1]) ** 2) / dWb   # dW in bins
        prev = omega[j - 1]
        cur = omega[j]
        for b in np.nonzero(rho)[0]:
            # trunc(w + f) is w + floor(f) where w + f >= 0 and w + ceil(f) where w + f < 0:
            # two runs of source bins, each moved by one integer shift
            first_up = int(np.ceil(-f[b]))            # smallest w with w + f >= 0
            for w_lo, w_hi, sh in ((first_up, M, int(np.floor(f[b]))), (-M, first_up - 1, int(np.ceil(f[b])))):
                lo, hi = max(w_lo, -M, -M - sh), min(w_hi, M, M - sh)
                if lo <= hi:
                    cur[lo + sh + M:hi + sh + M + 1] += rho[b] * prev[lo + M:hi + M + 1]
        cur[M] = 0.5 * (cur[M - 1] + cur[M + 1])
    je = np.full(s, np.nan)
    for j in range(s):
        tot = omega[j].sum()
        if tot > 0:
            je[j] = -kT * np.log(np.sum(omega[j] * np.exp(-beta * wv * dWb)) / tot)
    return {"work_hist_literal": omega, "dF_je_hist_literal": je}


def work_distributions_reverse(prob, hist, n, omega_fwd):
    """The reverse path lambda_j -> lambda_1 (Sec. V: forward and reverse work
    distributions; Crooks fluctuation theorem; Kofke's overlap).  Omega^rev_j is
    built like Omega_j, each step i+1 -> i from the x distribution of the window
    it starts from, rho_{i+1}, with the work of moving the centre back,
    dW^rev_i(x) = k/2 [(x - lambda_i)^2 - (x - lambda_{i+1})^2] at the bin centre,
    floor to bins.  After j folds (0-based j) a work bin w holds work in
    [w, w + j) dW in either direction, so the forward bin w and the reverse
    bin -w - j cover opposite intervals.  From them:
      dF_rev_hist_j = +kT ln sum_v Omega^rev_j(v) exp(-beta v dW) / sum Omega^rev_j
        (reverse JE: <exp(-beta W_rev)> = exp(+beta dF_j));
      crooks_ovl_j = sum_w min(Omega_j(w), Omega^rev_j(-w - j));
      dF_crooks_j: Crooks' P_f(W) / P_r(-W) = exp(beta (W - dF)) read in every bin
        both distributions hold, dF = W - kT ln(P_f / P_r) with W at the middle
        (w + j/2) dW of the common interval, averaged with weights
        min(P_f, P_r)."""
    lam = np.asarray(prob["lambda"], dtype=np.float64)
    s = len(lam)
    k = float(prob["k"]); kT = float(prob["kT"]); beta = 1.0 / kT
    M = int(prob["w_half_bins"]); dWb = float(prob["w_bin"])
    K = int(prob["xi_nbins"]); x0 = float(prob["xi_min"]); dx = float(prob["xi_bin"])
    nb = 2 * M + 1
    xb = x0 + (np.arange(K) + 0.5) * dx
    omega = np.zeros((s, nb))
    omega[0, M] = 1.0
    for j in range(1, s):
        rho = hist[j] / max(int(n[j]), 1)                 # the step lambda_j -> lambda_{j-1}
        dW = 0.5 * k * ((xb - lam[j - 1]) ** 2 - (xb - lam[j]) ** 2)
        shifts = np.floor(dW / dWb).astype(np.int64)
        prev = omega[j - 1]
        cur = omega[j]
        for b in np.nonzero(rho)[0]:
            sb = int(shifts[b])
            lo = max(0, -sb); hi = min(nb, nb - sb)
            if lo < hi:
                cur[lo + sb:hi + sb] += rho[b] * prev[lo:hi]
    wv = np.arange(-M, M + 1, dtype=np.float64)
    rev = np.full(s, np.nan); ovl = np.full(s, np.nan); crooks = np.full(s, np.nan)
    for j in range(s):
        tot = omega[j].sum()
        if tot > 0:
            rev[j] = kT * np.log(np.sum(omega[j] * np.exp(-beta * wv * dWb)) / tot)
        pf = omega_fwd[j]
        pr = np.zeros(nb)                                 # pr[w + M] = Omega^rev_j(-w - j)
        for w in range(-M, M + 1):
            v = -w - j
            if -M <= v <= M:
                pr[w + M] = omega[j][v + M]
        m = np.minimum(pf, pr)
        ovl[j] = m.sum()
        both = (pf > 0) & (pr > 0)
        if np.any(both):
            W = (wv[both] + 0.5 * j) * dWb
            crooks[j] = np.sum(m[both] * (W - kT * np.log(pf[both] / pr[both]))) / np.sum(m[both])
    return {"work_hist_rev": omega, "dF_rev_hist": rev, "crooks_ovl": ovl, "dF_crooks": crooks}


def product_form(prob, hist, n):
    """The exact exponential average of the binned x distributions, without work binning:
    -kT sum_{i<j} ln sum_b rho_i(b) exp(-beta dW_i(x_b)).  Used to pin the recursion."""
    lam = np.asarray(prob["lambda"], dtype=np.float64)
    k = float(prob["k"]); kT = float(prob["kT"]); beta = 1.0 / kT
    K = int(prob["xi_nbins"])
    x0 = float(prob["xi_min"]); dx = float(prob["xi_bin"])
    xb = x0 + (np.arange(K) + 0.5) * dx
    out = np.zeros(len(lam))
    for j in range(1, len(lam)):
        i = j - 1
        rho = hist[i] / max(int(n[i]), 1)
        dW = 0.5 * k * ((xb - lam[i + 1]) ** 2 - (xb - lam[i]) ** 2)
        out[j] = out[j - 1] - kT * np.log(np.sum(rho * np.exp(-beta * dW)) / np.sum(rho))
    return out
