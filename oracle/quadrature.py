"""Exact restrained free energies by quadrature and closed forms -- TEST INFRASTRUCTURE ONLY.

The profile the protocol estimates is dF(lambda_j) = F(lambda_j, k) - F(lambda_1, k)
with F(lambda, k) = -kT ln Z(lambda, k) and Z the configurational partition
function of H_o plus the restraint k/2 (x - lambda)^2 (Eq. 12 and the text
after it; the reference point F(lambda_1, k) is the one of Sec. IV A).  For the
systems below Z is a low-dimensional integral, done here by Gauss-Legendre
quadrature; the same integrals give <x>_lambda and sigma_lambda, from which the
expectations of the approximate estimators of Eqs. 13 and 14 follow.
"""
import numpy as np


def _gl(a, b, n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _panels(a, b, n_panels, order=64):
    xs, ws = [], []
    edges = np.linspace(a, b, n_panels + 1)
    for lo, hi in zip(edges[:-1], edges[1:]):
        x, w = _gl(lo, hi, order)
        xs.append(x); ws.append(w)
    return np.concatenate(xs), np.concatenate(ws)


def _moments(x, w, logp):
    """ln Z, <x>, var(x) of the density exp(logp) on nodes x with weights w."""
    m = np.max(logp)
    p = np.exp(logp - m) * w
    Z = p.sum()
    mean = np.sum(p * x) / Z
    var = np.sum(p * (x - mean) ** 2) / Z
    return m + np.log(Z), mean, var


def restrained_1d(U, lam, k, kT, lo=-4.0, hi=4.0, n_panels=4000):
    """F(lambda,k), <x>_lambda, var_lambda(x) for one particle in U(x) (arrays over lambda)."""
    x, w = _panels(lo, hi, n_panels)
    beta = 1.0 / kT
    Ux = U(x)
    F = []; mu = []; var = []
    for L in np.atleast_1d(lam):
        lz, m, v = _moments(x, w, -beta * (Ux + 0.5 * k * (x - L) ** 2))
        F.append(-kT * lz); mu.append(m); var.append(v)
    return np.array(F), np.array(mu), np.array(var)


def double_well(a=5.0, b=1.0):
    return lambda x: a * (x * x - b) ** 2


def harmonic_closed_form(kappa, k, kT, lam):
    """H_o = kappa/2 x^2 with the restraint: x ~ N(k lam/(kappa+k), kT/(kappa+k)),
    F(lambda) - F(0) = kappa k lam^2 / (2 (kappa + k))."""
    lam = np.asarray(lam, dtype=np.float64)
    mean = k * lam / (kappa + k)
    var = np.full_like(lam, kT / (kappa + k))
    F = kappa * k * lam ** 2 / (2.0 * (kappa + k))
    return F, mean, var


def chain2(lam, k, kT, k_bond, r0, lo=1e-6, hi=None, n_panels=2000):
    """Two beads, bead 0 fixed, xi = |r_1|: Z = int 4 pi r^2 exp(-beta[k_b/2 (r-r0)^2 + k/2 (r-lam)^2]) dr."""
    beta = 1.0 / kT
    lam_arr = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    if hi is None:
        hi = max(r0, lam_arr.max()) + 12.0 * np.sqrt(kT / min(k_bond, k)) + 1.0
    r, w = _panels(lo, hi, n_panels)
    F = []; mu = []; var = []
    for L in lam_arr:
        logp = 2.0 * np.log(r) - beta * (0.5 * k_bond * (r - r0) ** 2 + 0.5 * k * (r - L) ** 2)
        lz, m, v = _moments(r, w, logp)
        F.append(-kT * lz); mu.append(m); var.append(v)
    return np.array(F), np.array(mu), np.array(var)


def chain3(lam, k, kT, k_bond, r0, k_angle, n_b=96, n_c=192, width=8.0):
    """Three beads (no Lennard-Jones pair has |i-j| > 2), bead 0 fixed, xi = |r_2|.
    Bond lengths b1, b2 and c = cos(phi) of the angle between the bond vectors:
    xi^2 = b1^2 + b2^2 + 2 b1 b2 c, measure b1^2 db1 b2^2 db2 dc (the remaining
    orientation angles integrate to a constant)."""
    beta = 1.0 / kT
    sd = np.sqrt(kT / k_bond)
    blo = max(1e-6, r0 - width * sd); bhi = r0 + width * sd
    b, wb = _panels(blo, bhi, 4, n_b // 4)
    c, wc = _panels(-1.0, 1.0, 8, n_c // 8)
    B1, B2, C = np.meshgrid(b, b, c, indexing="ij")
    W = wb[:, None, None] * wb[None, :, None] * wc[None, None, :]
    xi = np.sqrt(np.maximum(B1 ** 2 + B2 ** 2 + 2.0 * B1 * B2 * C, 0.0))
    base = (2.0 * np.log(B1) + 2.0 * np.log(B2)
            - beta * (0.5 * k_bond * (B1 - r0) ** 2 + 0.5 * k_bond * (B2 - r0) ** 2 + k_angle * (1.0 - C)))
    F = []; mu = []; var = []
    for L in np.atleast_1d(np.asarray(lam, dtype=np.float64)):
        lz, m, v = _moments(xi.ravel(), W.ravel(), (base - beta * 0.5 * k * (xi - L) ** 2).ravel())
        F.append(-kT * lz); mu.append(m); var.append(v)
    return np.array(F), np.array(mu), np.array(var)


def estimator_expectations(lam, mu, var, k, kT):
    """Expected profiles of Eq. 14 and Eq. 13 (actual increments) when <x_i> and sigma_i
    take their exact values."""
    lam = np.asarray(lam, dtype=np.float64)
    s = len(lam)
    fl = np.zeros(s); g = np.zeros(s)
    for j in range(1, s):
        i = j - 1
        dl = lam[i + 1] - lam[i]
        fl[j] = fl[j - 1] + k * dl * (lam[i] - mu[i])
        g[j] = g[j - 1] + k * dl * (lam[i] - mu[i]) + 0.5 * k * dl * dl * (1.0 - k * var[i] / kT)
    return fl, g


def estimator_expectations_literal(lam, mu, var, k, kT):
    """The same for Eqs. 14 and 13 as printed: (lambda_j - lambda_1)/j per step up to lambda_j."""
    lam = np.asarray(lam, dtype=np.float64)
    s = len(lam)
    fl = np.zeros(s); g = np.zeros(s)
    for j in range(1, s):
        span = lam[j] - lam[0]
        fl[j] = k * span * np.sum(lam[:j] - mu[:j]) / (j + 1)
        g[j] = k * span ** 2 / (2.0 * (j + 1)) * np.sum(1.0 - k * np.asarray(var[:j]) / kT) / (j + 1) + fl[j]
    return fl, g


def turn_on_1d(U, lam, k, kT, lo=-4.0, hi=4.0, n_panels=4000):
    """Turn-on free energy dF(lambda, k) = F(lambda, k) - F_0 of one particle in U(x)
    (Eqs. 5-6, with F_0 = -kT ln int exp(-beta U)), and the two sides of Eq. 7:
    <k/2 (x - lambda)^2> over the restrained and over the unrestrained density."""
    x, w = _panels(lo, hi, n_panels)
    beta = 1.0 / kT
    Ux = U(x)
    lz0, m0, v0 = _moments(x, w, -beta * Ux)
    lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    F, mu, var = restrained_1d(U, lam, k, kT, lo, hi, n_panels)
    dF = F + kT * lz0
    lower = 0.5 * k * (var + (mu - lam) ** 2)
    upper = 0.5 * k * (v0 + (m0 - lam) ** 2)
    return dF, lower, upper


def harmonic_turn_on_closed_form(kappa, k, kT, lam):
    """dF(lambda, k) for H_o = kappa/2 x^2: the ratio of two Gaussian integrals,
    kT/2 ln((kappa + k)/kappa) + kappa k lambda^2 / (2 (kappa + k))."""
    lam = np.asarray(lam, dtype=np.float64)
    return 0.5 * kT * np.log((kappa + k) / kappa) + kappa * k * lam ** 2 / (2.0 * (kappa + k))


def chain2_turn_on(lam, k, kT, k_bond, r0, lo=1e-6, hi=None, n_panels=2000):
    """Turn-on free energy dF(lambda, k) = -kT ln [Z(lambda, k) / Z(0)] of the two-bead
    chain (bead 0 fixed, xi = |r_1|), both partition functions as radial integrals
    int 4 pi r^2 exp(-beta [k_b/2 (r - r0)^2 (+ k/2 (r - lambda)^2)]) dr."""
    beta = 1.0 / kT
    lam_arr = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    if hi is None:
        hi = max(r0, lam_arr.max()) + 12.0 * np.sqrt(kT / min(k_bond, k)) + 1.0
    r, w = _panels(lo, hi, n_panels)
    lz0, _, _ = _moments(r, w, 2.0 * np.log(r) - beta * 0.5 * k_bond * (r - r0) ** 2)
    F, _, _ = chain2(lam_arr, k, kT, k_bond, r0, lo, hi, n_panels)
    return F + kT * lz0
