"""Final dF of GPU runs against exact quadrature of the restrained partition
function (needs an MI355X): the 1-D double-well workload at full size, and the
chains with N = 2 and N = 3 beads, where no Lennard-Jones pair exists and the
radial (N = 2) or three-dimensional (N = 3) integral is exact.  JE is unbiased
up to sampling and time-step error, so it must land within 3 jackknife
standard errors; fp32 forces with fp64 accumulation are held to the same bar."""
import sys

import numpy as np
import pytest

import paper_1105_4840_amd as ppp
import ppp_inputs
from oracle import quadrature

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _z(res, exact):
    return (res["dF_je"][1:] - exact[1:]) / res["dF_je_se"][1:]


def test_double_well_workload_against_quadrature():
    """21 windows x 256 replicas x 20000 LM steps, fp64 (the 1-D workload itself)."""
    _say("case quadrature 1d workload")
    prob = ppp_inputs.config_1d()
    prob["n_blocks"] = 16
    res, _ = ppp.run(prob)
    F, mu, var = quadrature.restrained_1d(quadrature.double_well(), prob["lambda"], prob["k"], prob["kT"])
    exact = F - F[0]
    z = _z(res, exact)
    _say(f"  dF_je end {res['dF_je'][-1]:.4f} +- {res['dF_je_se'][-1]:.4f} (exact {exact[-1]:.4f}); max |z| {np.max(np.abs(z)):.2f}")
    assert abs(z[-1]) < 3.0 and np.max(np.abs(z)) < 4.0
    # window moments against the exact ones
    zm = (res["xi_mean"] - mu) / (res["xi_std"] / np.sqrt(res["n_samples"] / 10.0))
    assert np.max(np.abs(zm)) < 5.0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n_beads", [2, 3])
def test_short_chains_against_quadrature(n_beads, precision):
    _say(f"case quadrature chain N={n_beads} {precision}")
    prob = ppp_inputs.config_chain_small(n_beads, n_replicas=512, n_steps=20000, n_windows=8, precision=precision)
    prob["lambda"] = list(np.linspace(0.6, 1.6, 8) if n_beads == 2 else np.linspace(1.2, 2.2, 8))
    prob["n_blocks"] = 32
    prob["w_half_bins"] = 0
    res, _ = ppp.run(prob)
    if n_beads == 2:
        F, mu, var = quadrature.chain2(prob["lambda"], prob["k"], prob["kT"], prob["k_bond"], prob["r0"])
    else:
        F, mu, var = quadrature.chain3(prob["lambda"], prob["k"], prob["kT"], prob["k_bond"], prob["r0"], prob["k_angle"])
    exact = F - F[0]
    z = _z(res, exact)
    _say(f"  dF_je end {res['dF_je'][-1]:.4f} +- {res['dF_je_se'][-1]:.4f} (exact {exact[-1]:.4f}); "
         f"z {np.round(z, 2)}")
    assert abs(z[-1]) < 3.0 and np.max(np.abs(z)) < 3.5
    # Eq. 13 with exact moments is what dF_gauss estimates; its sampled value sits near it
    fl, g = quadrature.estimator_expectations(prob["lambda"], mu, var, prob["k"], prob["kT"])
    assert abs(res["dF_gauss"][-1] - g[-1]) < 3.0 * res["dF_gauss_se"][-1] + 1e-3


def test_crooks_estimate_matches_quadrature_on_1d_workload():
    """Forward and reverse path work distributions (App. C) on the 1-D workload:
    the Crooks estimate, which reads P_f(W) / P_r(-W) = exp(beta (W - dF)) in
    every bin both hold, against the exact profile; the one-sided histogram
    estimates are off by their left-edge binning (about j dW / 2 each way)."""
    print("case crooks 1d", flush=True)
    p = ppp_inputs.config_1d(n_replicas=256, n_steps=20000, precision="fp64")
    res, _ = ppp.run(p)
    F, _, _ = quadrature.restrained_1d(quadrature.double_well(), p["lambda"], p["k"], p["kT"])
    exact = F - F[0]
    err = res["dF_crooks"] - exact
    print("  crooks - exact", np.round(err, 4), flush=True)
    print("  overlap", np.round(res["crooks_ovl"], 3), flush=True)
    assert np.all(np.abs(err[1:]) < 4.0 * res["dF_je_se"][1:] + 0.01)
    s = len(p["lambda"])
    j = np.arange(s)
    dWb = p["w_bin"]
    assert np.all(np.abs(res["dF_rev_hist"] - exact) < 4.0 * res["dF_je_se"] + j * dWb + 0.01)
    assert res["crooks_ovl"][0] == 1.0 and res["crooks_ovl"][-1] < res["crooks_ovl"][1] < 1.0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_baoab_harmonic_position_variance_is_exact(precision):
    """The kernels' BAOAB with the chain's noise against a closed form: a
    two-bead chain with no bond, the projection reaction coordinate (xi = z_1 -
    z_0) and the restraint as the only force is a harmonic oscillator in z with
    K = k, whose sampled position variance BAOAB gets exactly, kT/K, at any
    stable step.  At k dt^2/4 = 0.45 other splittings are far off (ABOBA: 1.82
    kT/K), and a noise amplitude off by a factor (1 + e) moves the variance by
    (1 + e)^2.  16 windows x 4096 replicas x 1000 samples; every window has the
    same variance, so the spread of the 16 window variances gives the error of
    their mean whatever the samples' correlation."""
    k, dt, R, S = 20.0, 0.3, 4096, 16
    p = ppp_inputs.config_chain_small(2, n_replicas=R, n_steps=21000, n_windows=S, seed=9, precision=precision)
    lam = np.linspace(-1.0, 1.0, S)
    p.update({"k_bond": 0.0, "k_angle": 0.0, "lj_eps": 0.0, "rc_mode": 1, "k": k, "dt": dt,
              "lambda": lam.tolist(), "init_coords": [0.0, 0.0, 0.0, 1.0, 0.0, 0.25],
              "n_equil": 1000, "sample_every": 20})
    p.update(ppp_inputs._hist_spec(-4.0, 4.0, 1024))
    _say(f"case BAOAB harmonic variance {precision}: {S} windows x {R} replicas, k dt^2/4 = {k * dt * dt / 4:.2f}")
    res, _ = ppp.run(p)
    assert int(res["n_blown_up"].sum()) == 0
    assert np.all(res["n_samples"] == R * 1000)
    var = np.asarray(res["xi_std"]) ** 2
    mu = np.asarray(res["xi_mean"])
    want = p["kT"] / k
    se = var.std(ddof=1) / np.sqrt(S)
    _say(f"  mean variance {var.mean():.6f} (kT/k = {want:.6f}, se {se:.1e}); "
         f"max |mean - lambda| {np.max(np.abs(mu - lam)):.1e}")
    assert abs(var.mean() - want) < 4 * se
    assert abs(var.mean() - want) < 2e-3 * want
    # each window alone, against a 1% band (about eight times its own error)
    assert np.all(np.abs(var - want) < 0.01 * want)
    assert np.all(np.abs(mu - lam) < 5e-3)


@pytest.mark.parametrize("integrator,name", [(0, "LM"), (1, "EM")])
def test_overdamped_harmonic_variance_closed_form(integrator, name):
    """The 1-D kernel's overdamped schemes against closed forms on a harmonic
    well of total stiffness K = kappa + k at K dt = 0.6: Leimkuhler-Matthews
    keeps the exact variance kT/K at any step; Euler-Maruyama samples
    kT/(K (1 - K dt/2)), here 1.43 kT/K.  16 windows x 4096 replicas; every
    window has the same variance, so the spread of the window variances gives
    the error of their mean."""
    K, dt, R, S = 30.0, 0.02, 4096, 16
    p = ppp_inputs.config_harmonic_1d(kappa=K - 10.0, k=10.0, n_replicas=R, n_steps=21000, seed=4)
    lam = np.linspace(-1.0, 1.0, S)
    p.update({"lambda": lam.tolist(), "dt": dt, "integrator_1d": integrator, "init_coords": [0.0],
              "n_equil": 1000, "sample_every": 20})
    p.update(ppp_inputs._hist_spec(-3.0, 3.0, 1024))
    _say(f"case overdamped harmonic variance {name}: {S} windows x {R} replicas, K dt = {K * dt:.2f}")
    res, _ = ppp.run(p)
    var = np.asarray(res["xi_std"]) ** 2
    mu = np.asarray(res["xi_mean"])
    want = p["kT"] / K if integrator == 0 else p["kT"] / (K * (1.0 - K * dt / 2.0))
    mean_want = p["k"] * lam / K
    se = var.std(ddof=1) / np.sqrt(S)
    _say(f"  mean variance {var.mean():.6f} (closed form {want:.6f}, se {se:.1e}); "
         f"max |mean - k lambda/K| {np.max(np.abs(mu - mean_want)):.1e}")
    assert abs(var.mean() - want) < 4 * se
    assert abs(var.mean() - want) < 2e-3 * want
    assert np.all(np.abs(var - want) < 0.01 * want)
    assert np.all(np.abs(mu - mean_want) < 5e-3)
