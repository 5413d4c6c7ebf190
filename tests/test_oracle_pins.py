"""Pins of the CPU oracle against things other than itself (no GPU needed).

Each test ties one part of the oracle to the paper's worked numbers, a closed
form, a symmetry, an independent implementation or brute force, so that a
dropped term, a wrong sign or index, or a transposed operand fails here.
"""
import json
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import ppp_inputs
from oracle import appc, estimators, quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TORCH_INC = None
try:
    import torch.utils.cpp_extension as _ce
    TORCH_INC = _ce.include_paths()[0]
except Exception:  # pragma: no cover
    pass

# --------------------------------------------------------------------------- Philox

_PHILOX_CPP = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    // PyTorch's engine: key = seed, counter = (offset lo, offset hi, subseq lo, subseq hi)
    at::philox_engine e(seed, c2 | (c3 << 32), c0 | (c1 << 32));
    unsigned a = e(), b = e(), c = e(), d = e();
    printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


@pytest.mark.skipif(TORCH_INC is None, reason="torch headers not found")
def test_philox_matches_pytorch_engine():
    """Philox4x32-10 (Salmon et al., SC'11) against PyTorch's independent header implementation."""
    rng = np.random.default_rng(11)
    cases = [(0, 0, 0, 0, 0), (0, 1, 0, 0, 0), (2 ** 64 - 1, 2 ** 32 - 1, 2 ** 32 - 1, 2 ** 32 - 1, 2 ** 32 - 1)]
    for _ in range(200):
        cases.append((int(rng.integers(0, 2 ** 63)),) + tuple(int(x) for x in rng.integers(0, 2 ** 32, 4)))
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.cpp"); exe = os.path.join(d, "p")
        open(src, "w").write(_PHILOX_CPP)
        subprocess.run(["g++", "-std=c++17", "-O1", "-I", TORCH_INC, src, "-o", exe], check=True)
        inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        seed = c[0]
        mine = oracle.philox([seed & 0xFFFFFFFF, seed >> 32], list(c[1:]))
        assert mine == [int(x) for x in line.split()], c


def test_normals_statistics():
    """Box-Muller normals: mean 0, variance 1, Gaussian tails (KS), no correlation between slots."""
    from scipy import stats
    z = np.array([oracle.normals4(5, g, n, 3, 0) for g in range(40) for n in range(250)])
    assert abs(z.mean()) < 4.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z.ravel(), "norm").pvalue > 1e-3
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(4))) < 5.0 / np.sqrt(z.shape[0])


def test_normals6_statistics():
    """The chain's six normals per block (21-bit uniforms, two beads per block):
    mean 0, variance 1, Gaussian (KS) in every slot, no correlation between any
    two slots (the two beads of a block among them), and |z| below the bound
    sqrt(44 ln 2) that the smallest uniform 2^-22 sets.  A wrong shift or mask
    in the bit fields gives uniforms outside (0, 1) or shared bits, which these
    checks catch."""
    from scipy import stats
    z = np.array([oracle.normals6(11, g, n, m, 0) for g in range(20) for n in range(100) for m in range(5)])
    assert np.all(np.isfinite(z)) and np.max(np.abs(z)) < np.sqrt(44 * np.log(2))
    assert abs(z.mean()) < 4.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / z.size)
    for k in range(6):
        assert stats.kstest(z[:, k], "norm").pvalue > 1e-3, k
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(6))) < 5.0 / np.sqrt(z.shape[0])
    # squares of the slots are uncorrelated too (a shared radius would show here)
    c2 = np.corrcoef((z ** 2).T)
    assert np.max(np.abs(c2 - np.eye(6))) < 5.0 * np.sqrt(3.0 / z.shape[0])


# --------------------------------------------------------------------------- forces


def _fd_forces(prob, r, lam, h=1e-6):
    f = np.zeros_like(r)
    for i in range(r.shape[0]):
        for c in range(3):
            rp = r.copy(); rm = r.copy()
            rp[i, c] += h; rm[i, c] -= h
            f[i, c] = -(oracle.chain_forces(prob, rp, lam)[0] - oracle.chain_forces(prob, rm, lam)[0]) / (2 * h)
    return f


@pytest.mark.parametrize("n_beads,rc_mode", [(10, 0), (13, 0), (7, 1)])
def test_chain_forces_are_minus_energy_gradient(n_beads, rc_mode):
    prob = ppp_inputs.chain_forcefield(n_beads)
    prob.update({"k": 20.0, "rc_mode": rc_mode})
    for r in ppp_inputs.random_chain_coords(n_beads, 3, seed=n_beads):
        lam = 0.6 * (n_beads - 1)
        _, _, f = oracle.chain_forces(prob, r, lam)
        fd = _fd_forces(prob, r, lam)
        assert np.max(np.abs(f - fd)) <= 1e-6 * max(1.0, np.max(np.abs(f)))


def test_chain_force_special_cases():
    base = ppp_inputs.chain_forcefield(4)
    base.update({"k": 0.0})
    # straight chain at bond length r0: no bond force, no angle force; LJ pair (0,3) at r = 3 > rc
    r = np.array([[0, 0, 0], [0, 0, 1.0], [0, 0, 2.0], [0, 0, 3.0]])
    e, parts, f = oracle.chain_forces(base, r, 0.0)
    assert np.allclose(parts, 0.0, atol=1e-14) and np.allclose(f, 0.0, atol=1e-12)
    # the only LJ pair (0,3) at the LJ minimum 2^(1/6) sigma: zero LJ force, energy -eps - U(rc)
    rmin = 2.0 ** (1.0 / 6.0)
    prob = dict(base, k_bond=0.0, k_angle=0.0)
    r = np.array([[0, 0, 0], [0.3, 0.1, 0.2], [0.7, -0.2, 0.1], [rmin, 0, 0]])
    e, parts, f = oracle.chain_forces(prob, r, 0.0)
    u_rc = 4.0 * (2.5 ** -12 - 2.5 ** -6)
    assert abs(parts[2] - (-1.0 - u_rc)) < 1e-13
    assert np.allclose(f[0], 0.0, atol=1e-12) and np.allclose(f[3], 0.0, atol=1e-12)
    # at r = sigma the LJ energy is 0 - U(rc); beyond the cutoff it is exactly 0
    r[3] = [1.0, 0, 0]
    assert abs(oracle.chain_forces(prob, r, 0.0)[1][2] - (-u_rc)) < 1e-13
    r[3] = [2.6, 0, 0]
    assert oracle.chain_forces(prob, r, 0.0)[1][2] == 0.0
    # restraint: energy k/2 (xi - lam)^2 and force -k (xi - lam) along r_{N-1}
    prob = dict(base, k=7.0, k_bond=0.0, k_angle=0.0, lj_eps=0.0)
    r = np.array([[0, 0, 0], [0, 0, 1.0], [0, 1.0, 1.0], [3.0, 4.0, 0.0]])
    e, parts, f = oracle.chain_forces(prob, r, 2.0)
    assert abs(parts[3] - 0.5 * 7.0 * 9.0) < 1e-13
    assert np.allclose(f[3], -7.0 * 3.0 * np.array([0.6, 0.8, 0.0]), atol=1e-13)
    # angle: right angle between bonds gives k_theta (1 - 0)
    prob = dict(base, k=0.0, k_bond=0.0, lj_eps=0.0)
    r = np.array([[0, 0, 0], [1.0, 0, 0], [1.0, 1.0, 0], [1.0, 1.0, 1.0]])
    assert abs(oracle.chain_forces(prob, r, 0.0)[1][1] - 2 * 5.0) < 1e-13


def test_default_helix_geometry():
    r = oracle.default_helix(10)
    b = np.linalg.norm(np.diff(r, axis=0), axis=1)
    assert np.allclose(b, 1.0, atol=1e-13)
    assert np.allclose(r[0], 0.0)
    d3 = np.linalg.norm(r[3:] - r[:-3], axis=1)
    assert d3.min() > 1.3                      # no Lennard-Jones overlap in the start state
    assert abs(r[-1, 2] - 0.395 * 9) < 1e-12


def test_pot1d_force():
    prob = ppp_inputs.config_1d()
    for x in [-1.7, -0.3, 0.0, 0.9, 1.4]:
        e, F = oracle.pot1d(prob, x, 0.45)
        h = 1e-6
        fd = -(oracle.pot1d(prob, x + h, 0.45)[0] - oracle.pot1d(prob, x - h, 0.45)[0]) / (2 * h)
        assert abs(F - fd) < 1e-6 * max(1, abs(F))
        assert abs(e - (5 * (x * x - 1) ** 2 + 25 * (x - 0.45) ** 2)) < 1e-12


# --------------------------------------------------------------------------- integrators


def _harmonic_var(integrator, dt, K=30.0, kT=1.0, R=256, steps=6000):
    prob = ppp_inputs.config_harmonic_1d(kappa=K - 10.0, k=10.0, n_replicas=R, n_steps=steps, seed=4)
    prob.update({"lambda": [0.0, 0.5], "dt": dt, "integrator_1d": integrator, "init_coords": [0.0],
                 "n_equil": 1000, "sample_every": 20})
    xi, kept, _ = oracle.run(prob)
    x = xi[:R]                                  # window lambda = 0
    return x.var(axis=1, ddof=1).mean(), x.var(axis=1, ddof=1).std() / np.sqrt(R)


def test_lm_stationary_variance_is_exact_for_harmonic():
    """Leimkuhler-Matthews keeps the exact stationary variance kT/K of a harmonic well."""
    K, dt = 30.0, 0.02                        # K dt = 0.6: a large step makes any bias visible
    v, se = _harmonic_var(0, dt, K)
    assert abs(v - 1.0 / K) < 4 * se + 1e-4


def test_em_stationary_variance_closed_form():
    """Euler-Maruyama on a harmonic well: var = kT / (K (1 - K dt / 2))."""
    K, dt = 30.0, 0.02
    v, se = _harmonic_var(1, dt, K)
    assert abs(v - 1.0 / (K * (1 - K * dt / 2))) < 4 * se + 1e-4
    assert v - 1.0 / K > 8 * se               # and it is visibly biased


def test_baoab_harmonic_position_variance_is_exact():
    """BAOAB samples the exact position variance kT/K of a harmonic oscillator at
    any stable step (a 2x2 Lyapunov fixed point; the momentum variance is
    kT (1 - K dt^2/4) instead).  A two-bead chain with no bond, the projection
    reaction coordinate (xi = z_1 - z_0) and the restraint as the only force is
    that oscillator in z with K = k.  At k dt^2/4 = 0.45 the other splittings are
    far off: ABOBA, for one, gives kT/(K (1 - K dt^2/4)) = 1.82 kT/K."""
    k, dt, R = 20.0, 0.3, 256
    p = ppp_inputs.config_chain_small(2, n_replicas=R, n_steps=21000, n_windows=2, seed=9)
    p.update({"k_bond": 0.0, "k_angle": 0.0, "lj_eps": 0.0, "rc_mode": 1, "k": k, "dt": dt,
              "lambda": [0.0, 0.5], "init_coords": [0.0, 0.0, 0.0, 1.0, 0.0, 0.25],
              "n_equil": 1000, "sample_every": 20})
    xi, kept, _ = oracle.run(p)
    assert np.all(kept == xi.shape[1])
    for w, lam in enumerate(p["lambda"]):
        x = xi[w * R:(w + 1) * R]
        v = x.var(axis=1, ddof=1)
        se_v = v.std(ddof=1) / np.sqrt(R)
        assert abs(v.mean() - p["kT"] / k) < 3 * se_v, (w, v.mean(), se_v)
        mu = x.mean(axis=1)
        assert abs(mu.mean() - lam) < 3 * mu.std(ddof=1) / np.sqrt(R), (w, mu.mean())
    assert 8 * se_v < p["kT"] / k * 0.82            # the ABOBA value would fail by far


def test_linear_pull_schedule_hand_case_1d():
    """Reading R15: the restraint centre moves linearly from xi(x_o) to lambda_i over
    the first n_pull steps and then stays; the force on the state after m steps
    uses the centre c_m = xi(x_o) + (lambda_i - xi(x_o)) m / n_pull (m < n_pull).
    With the noise switched off (kT = 1e-200) the overdamped harmonic particle
    follows x_{m+1} = x_m + dt (-kappa x_m - k (x_m - c_m)) with the centres
    listed by hand; after the pull it relaxes geometrically to k lambda/(kappa+k)."""
    kappa, k, dt, lam, x0 = 4.0, 20.0, 1e-3, 2.0, -1.0
    p = ppp_inputs.config_harmonic_1d(kappa=kappa, k=k, n_replicas=1, n_steps=60)
    p.update({"lambda": [0.5, lam], "init_coords": [x0], "kT": 1e-200, "n_pull": 8, "n_equil": 8, "dt": dt})
    tr = oracle.trajectory(p, 1, 0, 60)[:, 0]
    centres = [-1.0, -0.625, -0.25, 0.125, 0.5, 0.875, 1.25, 1.625] + [2.0] * 52
    x = [x0]
    for c in centres:
        x.append(x[-1] + dt * (-kappa * x[-1] - k * (x[-1] - c)))
    assert np.max(np.abs(tr - np.array(x))) < 1e-14
    fixed = k * lam / (kappa + k)
    geo = (x[8] - fixed) * (1 - dt * (kappa + k)) ** np.arange(53) + fixed
    assert np.max(np.abs(tr[8:] - geo)) < 1e-13
    # no pull: the centre sits at lambda_i from the first step
    q = dict(p, n_pull=0)
    tr0 = oracle.trajectory(q, 1, 0, 5)[:, 0]
    assert abs(tr0[1] - (x0 + dt * (-kappa * x0 - k * (x0 - lam)))) < 1e-15


def test_linear_pull_schedule_hand_case_chain():
    """The same schedule for a chain starts from the start state's reaction
    coordinate: two beads, no bond, xi = z_1 - z_0 = 1.5 at the start, the
    restraint the only force; with the noise off BAOAB moves z alone:
    v += dt/2 F; z += dt/2 v; v = e^{-gamma dt} v; z += dt/2 v; F = -k (z - c_m);
    v += dt/2 F, with c_m = 1.5 + (4 - 1.5) m/10 for m < 10, then 4."""
    k, dt, g = 20.0, 0.05, 1.0
    p = ppp_inputs.config_chain_small(2, n_replicas=1, n_steps=40, n_windows=2)
    p.update({"k_bond": 0.0, "k_angle": 0.0, "lj_eps": 0.0, "rc_mode": 1, "k": k, "dt": dt, "gamma": g,
              "kT": 1e-200, "lambda": [1.0, 4.0], "init_coords": [0.0, 0.0, 0.0, 0.3, -0.2, 1.5],
              "n_pull": 10, "n_equil": 10})
    tr = oracle.trajectory(p, 1, 0, 40)
    cm = [1.5, 1.75, 2.0, 2.25, 2.5, 2.75, 3.0, 3.25, 3.5, 3.75] + [4.0] * 31
    z, v = 1.5, 0.0
    f = -k * (z - cm[0])
    zs = [z]
    for m in range(1, 41):
        v += 0.5 * dt * f
        z += 0.5 * dt * v
        v *= np.exp(-g * dt)
        z += 0.5 * dt * v
        f = -k * (z - cm[m])
        v += 0.5 * dt * f
        zs.append(z)
    assert np.max(np.abs(tr[:, 5] - np.array(zs))) < 1e-13
    assert np.max(np.abs(tr[:, 3:5] - [0.3, -0.2])) < 1e-90       # x, y feel no force
    assert np.all(tr[:, :3] == 0.0)                                 # bead 0 is fixed


def test_pulled_harmonic_je_matches_closed_form():
    """A run with the pull (n_pull > 0, sampling after it) from a start state far
    outside the windows still gives the equilibrium profile: JE and Eq. 13
    against the closed form of the restrained harmonic oscillator within 3 SE."""
    p = ppp_inputs.config_harmonic_1d(n_replicas=256, n_steps=8000)
    p.update({"init_coords": [-3.0], "n_pull": 1500, "n_equil": 2000})
    xi, kept, _ = oracle.run(p)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    Fc, mu, var = quadrature.harmonic_closed_form(p["pot_kappa"], p["k"], p["kT"], p["lambda"])
    fl, g = quadrature.estimator_expectations(p["lambda"], mu, var, p["k"], p["kT"])
    for est, ref in (("dF_je", Fc - Fc[0]), ("dF_gauss", g)):
        z = (r[est][-1] - ref[-1]) / r[est + "_se"][-1]
        assert abs(z) < 3.0, (est, r[est][-1], ref[-1], r[est + "_se"][-1])
    zm = (r["xi_mean"] - mu) / (r["xi_std"] / np.sqrt(r["n_samples"] / 20.0))
    assert np.max(np.abs(zm)) < 4.0


def test_trajectory_matches_run_samples():
    """The parity hook replays the same replica as the full run."""
    prob = ppp_inputs.config_chain_small(6, n_replicas=4, n_steps=60)
    prob.update({"n_equil": 0, "sample_every": 1})
    xi, kept, _ = oracle.run(prob)
    tr = oracle.trajectory(prob, 2, 3, 60)
    r = tr[:, -3:]
    d = np.linalg.norm(r, axis=1)
    assert np.allclose(d[1:], xi[2 * 4 + 3, :60], rtol=0, atol=1e-13)


def test_nan_start_freezes_replica():
    prob = ppp_inputs.config_1d(n_replicas=4, n_steps=200)
    prob["init_coords"] = [float("nan")]
    xi, kept, _ = oracle.run(prob)
    assert np.all(kept == 0)
    res = estimators.estimate(prob, xi, kept, with_appc=False)
    assert np.all(res["n_blown_up"] == 4)


# --------------------------------------------------------------------------- quadrature


def test_quadrature_reproduces_harmonic_closed_form():
    kappa, k, kT = 4.0, 20.0, 1.3
    lam = np.linspace(-1, 1, 7)
    F, mu, var = quadrature.restrained_1d(lambda x: 0.5 * kappa * x * x, lam, k, kT)
    Fc, muc, varc = quadrature.harmonic_closed_form(kappa, k, kT, lam)
    assert np.allclose(F - F[3], Fc - Fc[3], atol=1e-11)
    assert np.allclose(mu, muc, atol=1e-12) and np.allclose(var, varc, rtol=1e-10)


def test_double_well_profile_symmetry():
    """U(x) = U(-x) and a symmetric window set: F(lambda) = F(-lambda), so dF(lambda_21) = 0."""
    p = ppp_inputs.config_1d()
    F, mu, var = quadrature.restrained_1d(quadrature.double_well(), p["lambda"], p["k"], p["kT"])
    assert np.allclose(F, F[::-1], atol=1e-11)
    assert np.allclose(mu, -mu[::-1], atol=1e-12)


def test_chain2_quadrature_reduces_to_closed_form_without_bond():
    """N = 2, k_b = 0: xi = |r| with density r^2 exp(-beta k/2 (r - lam)^2); for lam >> sd
    F(lam) - F(lam') = -2 kT ln(lam/lam') up to O(sd^2/lam^2)."""
    k, kT = 400.0, 1.0
    F, mu, var = quadrature.chain2([20.0, 40.0], k, kT, 0.0, 1.0, lo=1e-3, hi=45.0, n_panels=4000)
    exact = -2 * kT * np.log(40.0 / 20.0) - kT * (np.log(1 + kT / (k * 40 ** 2)) - np.log(1 + kT / (k * 20 ** 2)))
    assert abs((F[1] - F[0]) - exact) < 1e-8


# --------------------------------------------------------------------------- estimators


def test_step_work_is_eq9_summand():
    x = np.array([0.3, 1.7]); li, ln, k = 0.5, 1.25, 7.2
    # Eq. 9: k/2 (lambda_{i+1} - lambda_i)(lambda_{i+1} + lambda_i - 2 x_i)
    assert np.allclose(estimators.step_work(x, li, ln, k), 0.5 * k * (ln - li) * (ln + li - 2 * x))


def test_gaussian_windows_make_eq13_exact():
    """Exactly Gaussian xi (restrained harmonic oscillator) with known moments:
    Eq. 13 reproduces the exact profile for any dlambda; Eq. 14 misses
    sum k dlambda^2/2 (1 - k/(kappa+k)); JE is unbiased."""
    kappa, k, kT = 4.0, 20.0, 1.0
    lam = np.linspace(-1, 1, 11)
    Fc, mu, var = quadrature.harmonic_closed_form(kappa, k, kT, lam)
    fl, g = quadrature.estimator_expectations(lam, mu, var, k, kT)
    exact = Fc - Fc[0]
    assert np.allclose(g, exact, atol=1e-12)
    dl = np.diff(lam)
    miss = np.concatenate([[0], np.cumsum(0.5 * k * dl ** 2 * (1 - k / (kappa + k)))])
    assert np.allclose(fl, exact - miss, atol=1e-12)


def test_oracle_je_matches_harmonic_closed_form():
    p = ppp_inputs.config_harmonic_1d(n_replicas=256, n_steps=8000)
    xi, kept, _ = oracle.run(p)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    Fc, mu, var = quadrature.harmonic_closed_form(p["pot_kappa"], p["k"], p["kT"], p["lambda"])
    exact = Fc - Fc[0]
    fl, g = quadrature.estimator_expectations(p["lambda"], mu, var, p["k"], p["kT"])
    for est, ref in (("dF_je", exact), ("dF_gauss", g), ("dF_fluct", fl)):
        z = (r[est][-1] - ref[-1]) / r[est + "_se"][-1]
        assert abs(z) < 3.0, (est, r[est][-1], ref[-1], r[est + "_se"][-1])
    assert np.allclose(r["gamma2"], p["k"] / (p["k"] + p["pot_kappa"]), rtol=0.05)


def test_oracle_je_matches_double_well_quadrature():
    p = ppp_inputs.config_1d(n_replicas=256, n_steps=20000, seed=1)
    xi, kept, _ = oracle.run(p)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    F, mu, var = quadrature.restrained_1d(quadrature.double_well(), p["lambda"], p["k"], p["kT"])
    exact = F - F[0]
    z = (r["dF_je"] - exact)[1:] / r["dF_je_se"][1:]
    assert abs(z[-1]) < 3.0 and np.max(np.abs(z)) < 4.0
    # dF_fluct is biased by construction (the exact moments put it about -2 kT off at the end)
    fl, g = quadrature.estimator_expectations(p["lambda"], mu, var, p["k"], p["kT"])
    assert abs((r["dF_fluct"][-1] - fl[-1]) / r["dF_fluct_se"][-1]) < 3.0
    assert fl[-1] < -1.9


@pytest.mark.parametrize("n_beads", [2, 3])
def test_oracle_chain_je_matches_quadrature(n_beads):
    """BAOAB chains with no Lennard-Jones pair: JE against exact radial (N=2) or 3-D (N=3) quadrature."""
    p = ppp_inputs.config_chain_small(n_beads, n_replicas=128, n_steps=6000, n_windows=6)
    p["lambda"] = list(np.linspace(0.6, 1.6, 6) if n_beads == 2 else np.linspace(1.2, 2.2, 6))
    p["n_blocks"] = 16
    xi, kept, _ = oracle.run(p)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    if n_beads == 2:
        F, mu, var = quadrature.chain2(p["lambda"], p["k"], p["kT"], p["k_bond"], p["r0"])
    else:
        F, mu, var = quadrature.chain3(p["lambda"], p["k"], p["kT"], p["k_bond"], p["r0"], p["k_angle"])
    exact = F - F[0]
    z = (r["dF_je"] - exact)[1:] / r["dF_je_se"][1:]
    # the final dF at the stated 3 SE; the running maximum over the 5 correlated
    # profile points at 3.5 (a family of tests, not one)
    assert abs(z[-1]) < 3.0 and np.max(np.abs(z)) < 3.5, z
    zm = (r["xi_mean"] - mu) / (r["xi_std"] / np.sqrt(r["n_samples"] / 20.0))
    assert np.max(np.abs(zm)) < 4.0


def test_kish_and_lse_definitions():
    a = np.zeros(10)
    assert abs(estimators.logsumexp(a) - np.log(10)) < 1e-15
    assert abs(estimators.logsumexp(np.array([1000.0, 1000.0])) - (1000 + np.log(2))) < 1e-12
    assert estimators.logsumexp(np.zeros(0)) == -np.inf


# --------------------------------------------------------------------------- App. C


def test_paper_variance_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "je_variance_example.json")))
    kT = g["boltzmann_kcal_per_mol_K"] * g["temperature_K"]
    var = appc.paper_variance(g["sigma_w_kcal_per_mol"], g["Q"], kT)
    assert abs(var - g["paper_variance_approx"]) < 0.05
    assert abs(np.sqrt(var) - g["paper_sd_approx"]) < 0.05
    assert abs(var - 0.7085) < 5e-4


def _tiny_problem():
    p = {"lambda": [0.0, 0.4, 1.0], "k": 3.0, "kT": 0.8, "xi_min": -0.5, "xi_bin": 0.25,
         "xi_nbins": 5, "w_bin": 0.05, "w_half_bins": 200}
    hist = np.array([[1, 3, 0, 2, 1], [0, 2, 2, 1, 4], [5, 0, 0, 0, 1]])
    return p, hist, hist.sum(axis=1)


def test_appc_brute_force_tiny():
    """Enumerate every combination of x bins of windows 1 and 2: the work bin is
    floor(dW_1(x_a)/dW) + floor(dW_2(x_b)/dW) and its probability rho_1(a) rho_2(b)."""
    p, hist, n = _tiny_problem()
    out = appc.work_distributions(p, hist, n)
    M = p["w_half_bins"]; dWb = p["w_bin"]
    lam = p["lambda"]; k = p["k"]
    xb = p["xi_min"] + (np.arange(5) + 0.5) * p["xi_bin"]
    ref2 = np.zeros(2 * M + 1); ref3 = np.zeros(2 * M + 1)
    for a in range(5):
        wa = int(np.floor(0.5 * k * ((xb[a] - lam[1]) ** 2 - (xb[a] - lam[0]) ** 2) / dWb))
        ref2[M + wa] += hist[0, a] / n[0]
        for b in range(5):
            wb = int(np.floor(0.5 * k * ((xb[b] - lam[2]) ** 2 - (xb[b] - lam[1]) ** 2) / dWb))
            ref3[M + wa + wb] += hist[0, a] / n[0] * hist[1, b] / n[1]
    assert np.allclose(out["work_hist"][1], ref2, atol=1e-15)
    assert np.allclose(out["work_hist"][2], ref3, atol=1e-15)
    assert out["work_hist"][0, M] == 1.0


def test_appc_bounds_against_product_form():
    """Each of the j-1 floors rounds the work down by less than one bin, so
    dF_left <= dF_product <= dF_left + (j-1) dW, with dF_product the exact
    exponential average of the binned x distributions."""
    p = ppp_inputs.config_1d(n_replicas=64, n_steps=4000, seed=2)
    xi, kept, _ = oracle.run(p)
    hist, _ = estimators.histograms(xi, kept, p)
    n = np.array([kept[w * 64:(w + 1) * 64].sum() for w in range(21)])
    out = appc.work_distributions(p, hist, n)
    prod = appc.product_form(p, hist, n)
    j = np.arange(21)
    assert np.all(out["dF_je_hist"] <= prod + 1e-9)
    assert np.all(prod <= out["dF_je_hist"] + j * p["w_bin"] + 1e-9)
    assert np.max(np.abs(out["work_lost"])) < 1e-12
    # and against the unbinned JE: x binning moves each step's work by at most k |dl| dxi / 2
    r = estimators.estimate(p, xi, kept, with_appc=False)
    tol = np.cumsum(np.concatenate([[0], p["k"] * np.abs(np.diff(p["lambda"])) * p["xi_bin"] / 2]))
    assert np.all(np.abs(prod - r["dF_je"]) <= tol + 1e-9)


# --------------------------------------------------------------------------- statistics of the estimators


def _synthetic(samples_per_window, lam, k, kT, blocks, xi_bin=1e-3, xi_min=-10.0):
    """Problem and sample arrays for the estimators from given per-window samples
    (one sample per replica, so a jackknife block is a set of replicas)."""
    R = len(samples_per_window[0])
    xi = np.concatenate([np.asarray(s, dtype=np.float64) for s in samples_per_window])[:, None]
    kept = np.ones(len(xi), dtype=np.int64)
    p = {"lambda": list(lam), "k": k, "kT": kT, "n_replicas": R, "n_blocks": blocks,
         "xi_min": xi_min, "xi_bin": xi_bin, "xi_nbins": int(round(-2 * xi_min / xi_bin)), "w_half_bins": 0}
    return p, xi, kept


def test_jackknife_se_of_a_mean_is_the_standard_error():
    """dF_fluct of the second window is linear in the first window's mean, and the
    delete-one jackknife error of a sample mean is exactly s / sqrt(n)."""
    rng = np.random.default_rng(3)
    R = 50
    x1 = rng.normal(0.7, 0.3, R); x2 = rng.normal(1.1, 0.3, R)
    k, dl = 7.0, 0.5
    p, xi, kept = _synthetic([x1, x2], [0.5, 0.5 + dl], k, 1.0, blocks=R)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    assert abs(r["dF_fluct"][1] - k * dl * (0.5 - x1.mean())) < 1e-12
    assert abs(r["dF_fluct_se"][1] - k * dl * np.std(x1, ddof=1) / np.sqrt(R)) < 1e-12


def test_gaussian_samples_give_exact_forward_and_reverse_profiles():
    """Exact restrained-harmonic samples (x ~ N(k lam/(kappa+k), kT/(kappa+k))):
    forward JE, reverse JE and Eq. 13 converge to kappa k (lam_j^2 - lam_1^2) / (2 (kappa+k));
    the Kish fraction of a Gaussian exponent of variance v is exp(-v); the overlap of two
    equal-width Gaussians is 2 Phi(-|dmu| / (2 sigma))."""
    from scipy.stats import norm
    kappa, k, kT = 4.0, 20.0, 0.8
    lam = np.array([-0.3, -0.15, 0.0, 0.12, 0.3])
    Fc, mu, var = quadrature.harmonic_closed_form(kappa, k, kT, lam)
    rng = np.random.default_rng(11)
    R = 100000
    smp = [rng.normal(m, np.sqrt(v), R) for m, v in zip(mu, var)]
    p, xi, kept = _synthetic(smp, lam, k, kT, blocks=16, xi_bin=0.01)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    exact = Fc - Fc[0]
    for key in ("dF_je", "dF_gauss"):
        assert np.all(np.abs(r[key] - exact) <= 5 * r[key + "_se"] + 1e-12), (key, r[key] - exact)
    # reverse JE (no jackknife): its spread is that of the forward estimate in this symmetric case
    assert np.all(np.abs(r["dF_rev"] - exact) <= 5 * r["dF_je_se"] + 1e-3), r["dF_rev"] - exact
    beta = 1.0 / kT
    v = (beta * k * np.diff(lam)) ** 2 * var[:-1]
    assert np.allclose(r["kish_frac"][:-1], np.exp(-v), rtol=0.02), (r["kish_frac"], np.exp(-v))
    ovl = 2 * norm.cdf(-np.abs(np.diff(mu)) / (2 * np.sqrt(var[:-1])))
    assert np.allclose(r["overlap_ovl"], ovl, atol=0.01), (r["overlap_ovl"], ovl)
    assert np.allclose(r["gamma2"], k / (kappa + k), rtol=0.01)


def test_reach_criterion_hand_case():
    """Reach = end of the window's samples in the pulling direction minus their mean."""
    lam = [0.0, 1.0, 3.0]
    smp = [[-1.0, 0.0, 1.0, 2.0], [0.0, 1.0, 1.0, 2.0], [2.0, 3.0, 3.0, 4.0]]
    p, xi, kept = _synthetic(smp, lam, 10.0, 1.0, blocks=2)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    assert np.allclose(r["reach"], [2.0 - 0.5, 2.0 - 1.0])
    assert np.allclose(r["dlambda_over_reach"], [1.0 / 1.5, 2.0 / 1.0])
    assert list(r["criterion_ok"]) == [True, False]
    # pulling towards smaller lambda measures the reach on the other side
    p2, xi2, kept2 = _synthetic(smp[::-1], lam[::-1], 10.0, 1.0, blocks=2)
    r2 = estimators.estimate(p2, xi2, kept2, with_appc=False)
    assert np.allclose(r2["reach"], [3.0 - 2.0, 1.0 - 0.0])


# --------------------------------------------------------------------------- sequential protocol (Sec. III(i))


def test_sequential_first_window_repeats_parallel_protocol():
    """Window 1 of the sequential protocol is the parallel protocol's window 1:
    same start, same restraint, same noise counters."""
    for p in (ppp_inputs.config_1d(n_replicas=12, n_steps=1500, n_windows=4),
              ppp_inputs.config_chain_small(7, n_replicas=6, n_steps=400, n_windows=3)):
        xi, kept, _ = oracle.run(p)
        xs, ks, _ = oracle.run(dict(p, sequential=True))
        R = p["n_replicas"]
        assert np.array_equal(xi[:R], xs[:R]) and np.array_equal(kept[:R], ks[:R])
        assert not np.array_equal(xi[R:], xs[R:])      # later windows start from the previous one


def test_sequential_harmonic_closed_form():
    p = dict(ppp_inputs.config_harmonic_1d(n_replicas=128, n_steps=6000), sequential=True)
    xi, kept, _ = oracle.run(p)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    Fc, mu, var = quadrature.harmonic_closed_form(p["pot_kappa"], p["k"], p["kT"], p["lambda"])
    z = (r["dF_je"][-1] - (Fc[-1] - Fc[0])) / r["dF_je_se"][-1]
    assert abs(z) < 3.0, z


def test_sequential_double_well_quadrature():
    p = dict(ppp_inputs.config_1d(n_replicas=128, n_steps=10000, seed=4), sequential=True)
    xi, kept, _ = oracle.run(p)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    F, mu, var = quadrature.restrained_1d(quadrature.double_well(), p["lambda"], p["k"], p["kT"])
    z = (r["dF_je"] - (F - F[0]))[1:] / r["dF_je_se"][1:]
    assert abs(z[-1]) < 3.0 and np.max(np.abs(z)) < 4.0, z


def test_sequential_frozen_replica_stays_frozen():
    p = dict(ppp_inputs.config_chain_small(5, n_replicas=3, n_steps=100, n_windows=3), sequential=True)
    init = ppp_inputs.random_chain_coords(5, 1, seed=2)[0]
    init[2, 0] = np.nan
    p["init_coords"] = init.ravel().tolist()
    xi, kept, _ = oracle.run(p)
    assert np.all(kept == 0)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    assert np.all(r["n_blown_up"] == 3)


# --------------------------------------------------------------------------- paper-literal readings


def test_literal_eq14_on_uniform_windows_and_double_well_value():
    """With uniform windows, (lambda_j - lambda_1)/j (j counted from 1 at lambda_1,
    i.e. j+1 points up to index j) replaces the increment dl by j dl/(j+1), so
    Eq. 14 as printed is the increment form times j/(j+1).  On the double well
    with exact moments it gives -1.9125 kT at lambda = 1.5 (against -2.0081 for
    the increment form and exactly 0 for the free energy)."""
    rng = np.random.default_rng(5)
    lam = np.linspace(-1.0, 2.0, 13)
    mu = lam + rng.normal(0, 0.2, lam.size); var = rng.uniform(0.01, 0.05, lam.size)
    fl, g = quadrature.estimator_expectations(lam, mu, var, 30.0, 1.0)
    fl_l, g_l = quadrature.estimator_expectations_literal(lam, mu, var, 30.0, 1.0)
    j = np.arange(lam.size)
    assert np.allclose(fl_l, fl * j / (j + 1), atol=1e-12)
    p = ppp_inputs.config_1d()
    F, mu, var = quadrature.restrained_1d(quadrature.double_well(), p["lambda"], p["k"], p["kT"])
    fl, _ = quadrature.estimator_expectations(p["lambda"], mu, var, p["k"], p["kT"])
    fl_l, _ = quadrature.estimator_expectations_literal(p["lambda"], mu, var, p["k"], p["kT"])
    assert abs(fl[-1] - (-2.0081)) < 5e-4 and abs(fl_l[-1] - (-1.9125)) < 5e-4


def test_literal_estimators_match_their_expectations():
    """The sampled literal estimators sit on the closed form for Gaussian windows."""
    kappa, k, kT = 4.0, 20.0, 0.8
    lam = np.array([-0.3, -0.15, 0.0, 0.12, 0.3])
    Fc, mu, var = quadrature.harmonic_closed_form(kappa, k, kT, lam)
    rng = np.random.default_rng(13)
    smp = [rng.normal(m, np.sqrt(v), 50000) for m, v in zip(mu, var)]
    p, xi, kept = _synthetic(smp, lam, k, kT, blocks=8, xi_bin=0.01)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    fl_l, g_l = quadrature.estimator_expectations_literal(lam, mu, var, k, kT)
    assert np.allclose(r["dF_fluct_literal"], fl_l, atol=0.02)
    assert np.allclose(r["dF_gauss_literal"], g_l, atol=0.02)


def test_literal_work_binning_hand_case():
    """One occupied x bin per window makes every work value deterministic.
    Bin upper edges x = (b+1) dx, work in units of dW: f1 = dW_1(x)/dW = 2.7
    then f2 = -3.4.  As printed: w2 = trunc(2.7) = 2, w3 = trunc(2 - 3.4) = -1,
    then Omega_3(0) = (Omega_3(-1) + Omega_3(1))/2 = 1/2 (Omega_2(0) stays 0).
    Floor instead would give 2 and then 2 + floor(-3.4) = -2."""
    dWb, k = 0.1, 2.0
    # x bin 3 of width 0.5 from 0: upper edge x = 2.0; choose lambdas so that
    # k/2[(x - l2)^2 - (x - l1)^2] = 0.27 and then -0.34
    x = 2.0
    l1 = 0.0
    # k/2 (l2^2 - l1^2) - k x (l2 - l1) = 0.27  ->  l2^2 - 4 l2 - 0.27 = 0
    l2 = 2.0 - np.sqrt(4.0 + 0.27)
    # k/2 (l3^2 - l2^2) - k x (l3 - l2) = -0.34 -> l3^2 - 4 l3 - (l2^2 - 4 l2 - 0.34) = 0
    c = l2 ** 2 - 4 * l2 - 0.34
    l3 = 2.0 - np.sqrt(4.0 + c)
    p = {"lambda": [l1, l2, l3], "k": k, "kT": 1.0, "xi_min": 0.0, "xi_bin": 0.5, "xi_nbins": 6,
         "w_bin": dWb, "w_half_bins": 10}
    hist = np.zeros((3, 6), dtype=np.int64); hist[:, 3] = 7
    out = appc.work_distributions_literal(p, hist, hist.sum(axis=1))
    om = out["work_hist_literal"]; M = 10
    assert om[1, M + 2] == 1.0 and om[1].sum() == 1.0
    assert om[2, M - 1] == 1.0 and om[2, M] == 0.5 and om[2].sum() == 1.5
    expect = -np.log((np.exp(0.1) + 0.5) / 1.5)
    assert abs(out["dF_je_hist_literal"][2] - expect) < 1e-12
    # with the bin centre (x = 1.75) as representative: f = 2.37, -2.98, so w3 = trunc(2 - 2.98) = 0
    fc = [0.5 * k * ((1.75 - b) ** 2 - (1.75 - a) ** 2) / dWb for a, b in ((l1, l2), (l2, l3))]
    assert int(np.trunc(np.trunc(fc[0]) + fc[1])) == 0


# ---------------------------------------------------------------------------
# Turn-on free energy (Sec. II, Eqs. 5-7, 10, 15; App. A)

def test_turn_on_quadrature_matches_harmonic_closed_form():
    """dF(lambda, k) = F(lambda, k) - F_0 by quadrature against the ratio of two
    Gaussian integrals, and the two sides of Eq. 7 against their Gaussian
    moments: <(x - lambda)^2> = kT/(kappa + k) + (kappa lambda/(kappa + k))^2
    restrained, kT/kappa + lambda^2 free."""
    kappa, k, kT = 4.0, 2.0, 1.0
    lam = np.array([-1.0, -0.3, 0.0, 0.4, 1.2])
    dF, lower, upper = quadrature.turn_on_1d(lambda x: 0.5 * kappa * x * x, lam, k, kT)
    assert np.allclose(dF, quadrature.harmonic_turn_on_closed_form(kappa, k, kT, lam), rtol=0, atol=1e-10)
    assert np.allclose(lower, 0.5 * k * (kT / (kappa + k) + (kappa * lam / (kappa + k)) ** 2), atol=1e-10)
    assert np.allclose(upper, 0.5 * k * (kT / kappa + lam ** 2), atol=1e-10)
    # Eq. 7 holds strictly for the exact values (Jensen), here and for the double well
    assert np.all(lower < dF) and np.all(dF < upper)
    dF2, lo2, up2 = quadrature.turn_on_1d(quadrature.double_well(), np.linspace(-1.5, 1.5, 7), 20.0, kT)
    assert np.all(lo2 < dF2) and np.all(dF2 < up2)


def _free_run(prob):
    prob = dict(prob, free_ensemble=True, w_half_bins=0)
    xi, kept, _ = oracle.run(prob)
    return prob, estimators.estimate(prob, xi, kept, with_appc=False)


def test_turn_on_estimators_harmonic_closed_form():
    """Eq. 5 (restrained samples) and Eq. 6 (free samples) at lambda_1 and lambda_s
    against the closed form, G of Eq. 15 against F(lambda_j) - F(lambda_1) -
    dF(lambda_1), and Eq. 10's average against 1.  kappa > k keeps the variance
    of Eq. 5's average finite; the lambda range is not symmetric, so lambda_1 and
    lambda_s cannot be confused."""
    kappa, k, kT = 4.0, 2.0, 1.0
    base = ppp_inputs.config_harmonic_1d(kappa=kappa, k=k, n_replicas=96, n_steps=20000)
    base["lambda"] = list(np.linspace(-1.0, 0.4, 8))
    base["n_blocks"] = 16
    prob, r = _free_run(base)
    on = r["turn_on"]
    lam = np.asarray(prob["lambda"])
    ex = quadrature.harmonic_turn_on_closed_form(kappa, k, kT, lam)
    for key, want in (("eq5_first", ex[0]), ("eq6_first", ex[0]), ("eq5_last", ex[-1]), ("eq6_last", ex[-1])):
        assert abs(on[key] - want) < 4.0 * on[key + "_se"], (key, on[key], want, on[key + "_se"])
        assert on[key + "_se"] < 0.05
    assert abs(on["eq10_log"]) < 4.0 * on["eq10_log_se"]
    F, _, _ = quadrature.harmonic_closed_form(kappa, k, kT, lam)
    G_exact = (F - F[0]) - ex[0]
    assert np.all(np.abs(r["G"] - G_exact) < 4.0 * r["G_se"] + 1e-12)
    assert on["free_n"] == prob["n_replicas"] * oracle.samples_per_replica(prob)
    assert abs(on["free_mean"]) < 0.05 and abs(on["free_std"] - np.sqrt(kT / kappa)) < 0.02


def test_turn_on_estimators_obey_eq7_on_any_sample():
    """Jensen holds for sample averages too: kT ln mean(exp(beta u)) >= mean(u) and
    -kT ln mean(exp(-beta u)) <= mean(u), so Eq. 5's estimate is never below the
    lower bound and Eq. 6's never above the upper one, whatever the sample."""
    rng = np.random.default_rng(4)
    lam, k, kT = np.array([0.3, 0.9, 1.7]), 7.0, 0.6
    for _ in range(20):
        x1, xs, x0 = rng.normal(0.2, 0.5, 50), rng.normal(1.5, 0.3, 40), rng.normal(0.0, 1.0, 60)
        v = estimators.turn_on_values(x1, xs, x0, lam, k, kT, 0.0)
        assert v["eq5_first"] >= 0.5 * k * np.mean((x1 - lam[0]) ** 2)
        assert v["eq5_last"] >= 0.5 * k * np.mean((xs - lam[-1]) ** 2)
        assert v["eq6_first"] <= 0.5 * k * np.mean((x0 - lam[0]) ** 2)
        assert v["eq6_last"] <= 0.5 * k * np.mean((x0 - lam[-1]) ** 2)
    # one sample each: the averages are single terms, so Eqs. 5 and 6 equal the bounds
    v = estimators.turn_on_values(np.array([0.5]), np.array([2.0]), np.array([-0.1]), lam, k, kT, 0.0)
    assert np.isclose(v["eq5_first"], 0.5 * k * 0.2 ** 2) and np.isclose(v["eq6_last"], 0.5 * k * 1.8 ** 2)


def test_turn_on_estimators_double_well_quadrature():
    """A shallow double well, U = (x^2 - 1)^2 (barrier 1 kT), with k = 2: both
    estimates at both ends against quadrature, the bounds of Eq. 7 bracketing
    them, Eq. 10's average near 1.  Eq. 5's integrand is the unrestrained
    density itself, so it converges only when the restrained window visits the
    whole of it: here the restraint is soft and the barrier low, and the well
    curvature 8 exceeds k, which keeps the variance of that average finite."""
    base = ppp_inputs.config_1d(n_replicas=96, n_steps=20000, n_windows=11, seed=7)
    base.update({"k": 2.0, "pot_a": 1.0, "n_blocks": 16})
    base["lambda"] = list(np.linspace(-1.2, 0.9, 11))
    prob, r = _free_run(base)
    on = r["turn_on"]
    lam = np.asarray(prob["lambda"])
    dF, lower, upper = quadrature.turn_on_1d(quadrature.double_well(a=1.0), lam[[0, -1]], 2.0, 1.0)
    for key, want in (("eq5_first", dF[0]), ("eq6_first", dF[0]), ("eq5_last", dF[1]), ("eq6_last", dF[1])):
        assert abs(on[key] - want) < 4.0 * on[key + "_se"] + 0.01, (key, on[key], want, on[key + "_se"])
    assert abs(on["lower_first"] - lower[0]) < 0.05 and abs(on["upper_first"] - upper[0]) < 0.2
    assert on["lower_first"] < on["eq5_first"] and on["eq6_first"] < on["upper_first"]
    assert abs(on["eq10_log"]) < 4.0 * on["eq10_log_se"] + 0.01


# ---------------------------------------------------------------------------
# Reverse-path work distributions and the Crooks / Kofke checks (Sec. V)

def test_reverse_work_distribution_brute_force_tiny():
    """Enumerate every combination of x bins of windows 2 and 3 for the reverse
    path lambda_3 -> lambda_1: the work bin is floor(dW^rev_2(x_c)/dW) +
    floor(dW^rev_1(x_b)/dW) with dW^rev_i(x) = k/2 [(x - lambda_i)^2 -
    (x - lambda_{i+1})^2], its probability rho_2(b) rho_3(c)."""
    p, hist, n = _tiny_problem()
    fwd = appc.work_distributions(p, hist, n)
    out = appc.work_distributions_reverse(p, hist, n, fwd["work_hist"])
    M = p["w_half_bins"]; dWb = p["w_bin"]
    lam = p["lambda"]; k = p["k"]
    xb = p["xi_min"] + (np.arange(5) + 0.5) * p["xi_bin"]
    ref2 = np.zeros(2 * M + 1); ref3 = np.zeros(2 * M + 1)
    for b in range(5):
        wb = int(np.floor(0.5 * k * ((xb[b] - lam[0]) ** 2 - (xb[b] - lam[1]) ** 2) / dWb))
        ref2[M + wb] += hist[1, b] / n[1]
        for c in range(5):
            wc = int(np.floor(0.5 * k * ((xb[c] - lam[1]) ** 2 - (xb[c] - lam[2]) ** 2) / dWb))
            ref3[M + wb + wc] += hist[1, b] / n[1] * hist[2, c] / n[2]
    assert np.allclose(out["work_hist_rev"][1], ref2, atol=1e-15)
    assert np.allclose(out["work_hist_rev"][2], ref3, atol=1e-15)
    assert out["dF_rev_hist"][0] == 0.0 and out["crooks_ovl"][0] == 1.0 and out["dF_crooks"][0] == 0.0


def _gaussian_windows(kappa, k, kT, lam, dx, lo, hi):
    """Exact restrained densities of kappa/2 x^2 + k/2 (x - lambda)^2, integrated
    over bins of width dx (as counts out of 10^12), for the windows lam."""
    from scipy.special import erf
    edges = np.arange(lo, hi + dx / 2, dx)
    K = len(edges) - 1
    F, mu, var = quadrature.harmonic_closed_form(kappa, k, kT, lam)
    sd = np.sqrt(var)
    cdf = 0.5 * (1.0 + erf((edges[None, :] - mu[:, None]) / (np.sqrt(2.0) * sd[:, None])))
    n = 10 ** 12
    hist = np.diff(cdf, axis=1) * n
    return hist, np.full(len(lam), n, dtype=np.int64), F - F[0], K


def test_crooks_relation_on_exact_gaussian_windows():
    """With the exact restrained densities of a harmonic well in place of sampled
    histograms, every step's work is linear in x, the forward and reverse path
    work distributions are Gaussian, and Crooks' P_f(W) / P_r(-W) =
    exp(beta (W - dF)) holds exactly in the continuum: binned finely, the log
    ratio over the bins both distributions hold has slope beta in W and
    intercept -beta dF (the closed form), the reverse exponential average gives
    dF, and the overlap-weighted Crooks estimate gives dF."""
    kappa, k, kT = 4.0, 20.0, 0.7
    lam = np.linspace(-1.0, 0.6, 5)
    hist, n, dF, K = _gaussian_windows(kappa, k, kT, lam, 0.0005, -3.0, 3.0)
    M = 600; dWb = 0.02      # coarse work bins: a mirror off by j bins would move dF by j dW
    p = {"lambda": lam, "k": k, "kT": kT, "w_half_bins": M, "w_bin": dWb,
         "xi_nbins": K, "xi_min": -3.0, "xi_bin": 0.0005}
    fwd = appc.work_distributions(p, hist, n)
    rev = appc.work_distributions_reverse(p, hist, n, fwd["work_hist"])
    for j in range(1, len(lam)):
        pf = fwd["work_hist"][j]
        w = np.arange(-M, M + 1)
        v = -w - j
        ok = (v >= -M) & (v <= M)
        pr = np.zeros_like(pf); pr[ok] = rev["work_hist_rev"][j][v[ok] + M]
        both = (pf > 1e-6) & (pr > 1e-6)
        W = (w[both] + 0.5 * j) * dWb
        slope, icpt = np.polyfit(W, np.log(pf[both] / pr[both]), 1)
        assert abs(slope * kT - 1.0) < 0.02, (j, slope * kT)
        assert abs(-icpt / slope - dF[j]) < 0.02, (j, -icpt / slope, dF[j])
        assert abs(rev["dF_rev_hist"][j] - dF[j]) < 0.005 + j * dWb   # left-edge W: up to j dW
        assert abs(rev["dF_crooks"][j] - dF[j]) < 0.005
        assert 0.0 < rev["crooks_ovl"][j] <= 1.0
    # the overlap shrinks as the path gets longer
    assert np.all(np.diff(rev["crooks_ovl"][1:]) < 0)


# ---------------------------------------------------------------------------
# sigma_i by least-squares fitting (Sec. IV A)

def test_gauss_fit_recovers_an_exact_gaussian():
    """Histogram values that are exactly a Gaussian density at the bin centres:
    the least-squares fit returns its amplitude, centre and width."""
    dx, x0, K, n = 0.01, -2.0, 500, 10 ** 6
    x = x0 + (np.arange(K) + 0.5) * dx
    mu, sg = 0.137, 0.2315
    dens = np.exp(-(x - mu) ** 2 / (2 * sg ** 2)) / (sg * np.sqrt(2 * np.pi))
    A, m, s = estimators.gauss_fit(dens * n * dx, n, x0, dx, mu + 0.03, sg * 1.2)
    assert abs(m - mu) < 1e-10 and abs(s - sg) < 1e-10 and abs(A - 1 / (sg * np.sqrt(2 * np.pi))) < 1e-9


def test_gauss_fit_is_a_least_squares_minimum():
    """On a skewed histogram the fitted (A, mu, sigma) is a stationary point of
    the stated objective (central differences of the summed squared residual
    vanish to rounding) and beats the moments it starts from."""
    rng = np.random.default_rng(8)
    smp = np.concatenate([rng.normal(0.0, 0.3, 40000), rng.normal(0.6, 0.2, 15000)])
    dx, x0, K = 0.02, -2.0, 200
    counts = np.bincount(np.floor((smp - x0) / dx).astype(int), minlength=K)[:K]
    n = smp.size
    A, m, s = estimators.gauss_fit(counts, n, x0, dx, smp.mean(), smp.std(ddof=1))
    x = x0 + (np.arange(K) + 0.5) * dx
    y = counts / (n * dx)

    def cost(p):
        return np.sum((y - p[0] * np.exp(-(x - p[1]) ** 2 / (2 * p[2] ** 2))) ** 2)
    p = np.array([A, m, s])
    for q in range(3):
        h = 1e-6 * max(abs(p[q]), 1e-3)
        e = np.zeros(3); e[q] = h
        grad = (cost(p + e) - cost(p - e)) / (2 * h)
        assert abs(grad) < 1e-6 * (1 + cost(p) / abs(p[q])), (q, grad)
    start = np.array([1 / (smp.std(ddof=1) * np.sqrt(2 * np.pi)), smp.mean(), smp.std(ddof=1)])
    assert cost(p) < cost(start)
    # the same minimum as MINPACK's Levenberg-Marquardt from the same start
    from scipy.optimize import least_squares
    ref = least_squares(lambda q: y - q[0] * np.exp(-(x - q[1]) ** 2 / (2 * q[2] ** 2)), start, method="lm",
                        xtol=1e-15, ftol=1e-15, gtol=1e-15)
    assert np.allclose([A, m, s], [ref.x[0], ref.x[1], abs(ref.x[2])], rtol=1e-9)
    # a window without enough samples has no fit
    assert all(np.isnan(estimators.gauss_fit(np.zeros(5), 2, 0.0, 1.0, 0.0, 1.0)))


def test_turn_on_two_bead_chain_against_radial_quadrature():
    """The chain path of the unrestrained ensemble (BAOAB with the restraint off):
    for two beads, Eq. 5 and Eq. 6 at both ends against the ratio of the two radial
    partition functions.  The bond (k_b = 100) is stiffer than the restraint (k = 20),
    so the restrained windows cover the free density and Eq. 5's average has finite
    variance."""
    p = ppp_inputs.config_chain_small(2, n_replicas=64, n_steps=6000, n_windows=4, precision="fp64")
    p["lambda"] = [0.8, 0.95, 1.1, 1.25]
    p.update({"free_ensemble": True, "w_half_bins": 0, "n_blocks": 16})
    xi, kept, _ = oracle.run(p)
    r = estimators.estimate(p, xi, kept, with_appc=False)
    on = r["turn_on"]
    exact = quadrature.chain2_turn_on([0.8, 1.25], 20.0, 1.0, 100.0, 1.0)
    for key, want in (("eq5_first", exact[0]), ("eq6_first", exact[0]), ("eq5_last", exact[1]), ("eq6_last", exact[1])):
        assert abs(on[key] - want) < 4.0 * on[key + "_se"] + 0.005, (key, on[key], want, on[key + "_se"])
    assert abs(on["eq10_log"]) < 4.0 * on["eq10_log_se"] + 0.005
    # the free ensemble's end-to-end distance is the bond length distribution
    r_grid = np.linspace(0.5, 1.5, 20001)
    dens = r_grid ** 2 * np.exp(-50.0 * (r_grid - 1.0) ** 2)
    mean_exact = np.sum(r_grid * dens) / np.sum(dens)
    assert abs(on["free_mean"] - mean_exact) < 0.01
