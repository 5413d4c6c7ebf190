"""Learned window placement end to end (needs an MI355X): exploration rounds, GPU
training of the bf16 surrogate, placement by |dlambda|/sigma, production run."""
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


def test_adaptive_double_well_meets_overlap_target_and_quadrature():
    print("case adaptive 1d", flush=True)
    base = ppp_inputs.config_1d(n_replicas=256, n_steps=4000, precision="fp64")
    base["n_blocks"] = 16
    budget = 21 * 256 * 20000
    ad = {"budget_replica_steps": budget, "initial_windows": 11, "max_rounds": 4, "max_windows": 128,
          "target_dl_over_sigma": 1.0, "train_iters": 600, "lr": 3e-3, "init_seed": 3,
          "explore_replicas": 32, "explore_steps": 2000, "min_production_steps": 1000}
    res, lam, used = ppp.ppp_adaptive_run(base, ad)
    print(f"  windows {len(lam)}, used {used:.3g} of {budget:.3g}", flush=True)
    print("  dl/sigma", np.round(res["dlambda_over_sigma"], 2), flush=True)
    assert used <= budget and used > 0.9 * budget
    assert abs(lam[0] - (-1.5)) < 1e-12 and abs(lam[-1] - 1.5) < 1e-12 and np.all(np.diff(lam) > 0)
    # the placement follows sigma(lambda): narrower windows at the ends (sigma 0.09) than mid-way
    dl = np.diff(lam)
    assert dl[0] < 0.8 * np.max(dl)
    # overlap target met (measured sigma of the production run) better than 21 uniform windows
    assert np.max(res["dlambda_over_sigma"]) < 1.4
    F, mu, var = quadrature.restrained_1d(quadrature.double_well(), lam, base["k"], base["kT"])
    exact = F - F[0]
    z = (res["dF_je"][-1] - exact[-1]) / res["dF_je_se"][-1]
    print(f"  dF_je end {res['dF_je'][-1]:.4f} exact {exact[-1]:.4f} z {z:.2f}", flush=True)
    assert abs(z) < 3.5


def test_learned_placement_beats_uniform_windows_at_half_the_budget():
    """What the trained surrogate gains: with a stiff restraint (k = 800) the 21
    uniform windows of the double-well workload lie 4.5 sigma apart, their
    forward work distributions barely overlap and JE misses the exact
    dF(1.5) = 0 by several kT; placement by the surrogate at half the
    replica-steps lands within the statistical error."""
    print("case learned vs uniform 1d k=800", flush=True)
    base = ppp_inputs.config_1d(n_replicas=256, n_steps=20000, precision="fp64", seed=5)
    base["k"] = 800.0
    base["n_blocks"] = 16
    base["w_half_bins"] = 0
    budget = 21 * 256 * 20000
    uni, _ = ppp.run(base)
    err_u = abs(uni["dF_je"][-1])                     # exact: F(1.5) = F(-1.5) by symmetry
    ad = {"budget_replica_steps": budget // 2, "initial_windows": 11, "max_rounds": 5, "max_windows": 192,
          "target_dl_over_sigma": 1.0, "train_iters": 600, "lr": 3e-3, "init_seed": 3,
          "explore_replicas": 32, "explore_steps": 2000, "min_production_steps": 1000}
    res, lam, used = ppp.ppp_adaptive_run(dict(base, n_steps=4000), ad)
    err_l = abs(res["dF_je"][-1])
    print(f"  uniform: max dl/sigma {np.nanmax(uni['dlambda_over_sigma']):.2f}, |dF err| {err_u:.3f} "
          f"(se {uni['dF_je_se'][-1]:.3f}); learned: {len(lam)} windows, {used:.3g} replica-steps, "
          f"max dl/sigma {np.nanmax(res['dlambda_over_sigma']):.2f}, |dF err| {err_l:.3f} "
          f"(se {res['dF_je_se'][-1]:.3f})", flush=True)
    assert used <= budget // 2
    assert err_u > 1.0                                  # the uniform protocol fails here
    assert err_l < 0.25 * err_u
    assert err_l < 3.5 * res["dF_je_se"][-1] + 0.05
