"""GPU path against the CPU oracle, through the C ABI (needs an MI355X).

Deterministic parity: Philox words bit-exact; single-step forces and energies
(fp64 mode 1e-12, fp32 mode 1e-5, relative, norm-wise per configuration);
<= 100-step fp64 trajectories within 1e-10; whole fp64 runs: sample counts and
histograms exact, moments, log-sum-exp and profiles to 1e-9.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1105_4840_amd as ppp
import ppp_inputs
from oracle import estimators

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def test_philox_bits_and_normals():
    """Philox words against the oracle's; the four normals of a block (1-D model)
    and the six of the chain's noise in fp64 within 1e-13 of the oracle's.  fp32
    four-normal deviates differ by the 23-bit uniforms (2e-4 relative); the six
    fp32 normals use the oracle's 21-bit uniforms exactly, so only fp32 rounding
    of log2, the product, sqrt and sin/cos of 2 pi u separates them: well below
    1e-6 (1 + |z|) (9e-8 measured)."""
    _say("case philox")
    n = 4096
    worst = 0.0
    for seed, c1, c2, c3 in [(0, 0, 0, 0), (123456789012345, 7, 11, 0), (2 ** 64 - 1, 2 ** 32 - 1, 5, 9)]:
        w, z64, z32, y64, y32 = ppp.ppp_philox(seed, 1000, c1, c2, c3, n)
        for i in range(0, n, 97):
            ref = oracle.philox([seed & 0xFFFFFFFF, seed >> 32], [1000 + i, c1, c2, c3])
            assert [int(x) for x in w[i]] == ref
            zr = oracle.normals4(seed, 1000 + i, c1, c2, c3)
            assert np.max(np.abs(z64[i] - zr)) < 1e-13
            # fp32 deviates: 23-bit uniforms and hardware transcendentals
            assert np.max(np.abs(z32[i] - zr)) < 2e-4 * (1 + np.max(np.abs(zr)))
            yr = oracle.normals6(seed, 1000 + i, c1, c2, c3)
            assert np.max(np.abs(y64[i] - yr)) < 1e-13
            err = np.abs(y32[i] - yr) / (1 + np.abs(yr))
            worst = max(worst, float(np.max(err)))
            assert np.max(err) < 1e-6, (i, y32[i], yr)
    _say(f"  fp32 six-normal deviation: max |dz| / (1 + |z|) = {worst:.2e}")
    from scipy import stats
    for z in (z32, y32):
        assert abs(z.mean()) < 0.02 and abs(z.var() - 1) < 0.03
        assert stats.kstest(z.ravel(), "norm").pvalue > 1e-4
    assert np.max(np.abs(y32)) <= np.sqrt(44 * np.log(2)) + 1e-5


FORCE_CASES = [2, 3, 4, 9, 10, 13, 16, 23, 32, 37, 64, 100, 128, 200, 255, 256]


@pytest.mark.parametrize("n_beads", FORCE_CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_chain_forces(n_beads, precision):
    _say(f"case forces N={n_beads} {precision}")
    prob = ppp_inputs.config_chain_small(n_beads, n_replicas=4, n_steps=10, precision=precision)
    conf = ppp_inputs.random_chain_coords(n_beads, 5, seed=n_beads)
    lam = 0.6 * (n_beads - 1)
    h = ppp.ppp_create(prob)
    try:
        ws = ppp.workspace(h)
        x = torch.tensor(conf.reshape(len(conf), -1), dtype=torch.float64, device="cuda")
        f, e = ppp.ppp_eval_forces(h, ws, x, lam)
        f = f.cpu().numpy().reshape(len(conf), -1, 3); e = e.cpu().numpy()
    finally:
        ppp.ppp_destroy(h)
    tol = 1e-12 if precision == "fp64" else 1e-5
    for c in range(len(conf)):
        # the fp32 kernel works on the fp32-rounded coordinates: compare against the
        # exact forces of those coordinates, so only the kernel's arithmetic is measured
        xc = conf[c] if precision == "fp64" else conf[c].astype(np.float32).astype(np.float64)
        etot, parts, fr = oracle.chain_forces(prob, xc, lam)
        # bead 0 is held fixed: the kernel leaves the restraint's reaction
        # k (xi - lambda) dxi/dx_last off it (its bonded and LJ forces stay)
        want = fr.copy()
        end = xc[-1] - xc[0]
        if prob.get("rc_mode", 0) == 1:
            xi, dxi = end[2], np.array([0.0, 0.0, 1.0])
        else:
            xi = np.linalg.norm(end)
            dxi = end / xi
        want[0] -= prob["k"] * (xi - lam) * dxi
        d = f[c] - want
        assert np.linalg.norm(d) <= tol * np.linalg.norm(want), (c, np.linalg.norm(d), np.linalg.norm(want))
        assert np.linalg.norm(d[0]) <= tol * np.linalg.norm(want), (c, d[0])
        scale = np.sum(np.abs(parts)) + 1.0
        assert abs(e[c, 0] - etot) <= tol * scale
        assert np.all(np.abs(e[c, 1:] - parts) <= tol * scale)


def test_pot1d_forces():
    _say("case forces 1d")
    for precision, tol in (("fp64", 1e-13), ("fp32", 1e-5)):
        prob = ppp_inputs.config_1d(n_replicas=4, n_steps=10, precision=precision)
        xs = np.linspace(-2, 2, 33)
        h = ppp.ppp_create(prob)
        try:
            ws = ppp.workspace(h)
            f, e = ppp.ppp_eval_forces(h, ws, torch.tensor(xs[:, None], device="cuda", dtype=torch.float64), 0.3)
            f = f.cpu().numpy()[:, 0]; e = e.cpu().numpy()
        finally:
            ppp.ppp_destroy(h)
        for i, x in enumerate(xs):
            er, Fr = oracle.pot1d(prob, x, 0.3)
            assert abs(f[i] - Fr) <= tol * (1 + abs(Fr))
            assert abs(e[i, 0] - er) <= tol * (1 + abs(er))


@pytest.mark.parametrize("n_beads,window,replica", [(10, 1, 5), (13, 0, 3), (32, 2, 7), (37, 1, 2), (64, 3, 1),
                                                    (100, 1, 0), (256, 2, 1)])
def test_chain_trajectory_fp64(n_beads, window, replica):
    _say(f"case trajectory N={n_beads}")
    prob = ppp_inputs.config_chain_small(n_beads, n_replicas=8, n_steps=100, n_windows=4, precision="fp64")
    h = ppp.ppp_create(prob)
    try:
        ws = ppp.workspace(h)
        tr = ppp.ppp_trajectory(h, ws, window, replica, 100, 3 * n_beads).cpu().numpy()
    finally:
        ppp.ppp_destroy(h)
    ref = oracle.trajectory(prob, window, replica, 100)
    assert np.max(np.abs(tr - ref)) < 1e-10, np.max(np.abs(tr - ref))


def test_1d_trajectory_fp64():
    _say("case trajectory 1d")
    prob = ppp_inputs.config_1d(n_replicas=300, n_steps=100, precision="fp64")
    for integ in (0, 1):
        prob["integrator_1d"] = integ
        h = ppp.ppp_create(prob)
        try:
            ws = ppp.workspace(h)
            tr = ppp.ppp_trajectory(h, ws, 3, 260, 100, 1).cpu().numpy()
        finally:
            ppp.ppp_destroy(h)
        ref = oracle.trajectory(prob, 3, 260, 100)
        assert np.max(np.abs(tr - ref)) < 1e-10


def _compare_runs(prob, res, ref, prof_tol=1e-9):
    assert np.array_equal(res["n_samples"], ref["n_samples"])
    assert np.array_equal(res["n_blown_up"], ref["n_blown_up"])
    assert np.array_equal(res["xi_hist"].astype(np.int64), ref["xi_hist"])
    assert np.array_equal(res["xi_under_over"].astype(np.int64), ref["xi_under_over"])
    for key in ("xi_mean", "xi_std", "gamma2", "xi_min_sample", "xi_max_sample"):
        assert np.allclose(res[key], ref[key], rtol=1e-10, atol=1e-12, equal_nan=True), key
    s = len(prob["lambda"])
    assert np.allclose(res["lse_fwd"][:s - 1], ref["lse_fwd"][:s - 1], rtol=1e-11, atol=1e-9)
    assert np.allclose(res["lse_rev"][1:], ref["lse_rev"][1:], rtol=1e-11, atol=1e-9)
    for key in ("dF_je", "dF_fluct", "dF_gauss", "dF_com", "dF_unc", "dF_rev", "dF_fluct_literal", "dF_gauss_literal"):
        assert np.max(np.abs(res[key] - ref[key])) < prof_tol * (1 + np.max(np.abs(ref[key]))), key
    for key in ("dF_je_se", "dF_fluct_se", "dF_gauss_se", "dF_com_se"):
        assert np.allclose(res[key][1:], ref[key][1:], rtol=1e-7, atol=1e-12, equal_nan=True), key
    for key in ("kish_frac", "overlap_ovl", "dlambda_over_sigma", "dlambda_over_reach"):
        assert np.allclose(res[key], ref[key][:s - 1], rtol=1e-9, atol=1e-12), key
    assert np.array_equal(res["criterion_ok"].astype(bool), ref["criterion_ok"][:s - 1])
    # least-squares Gaussian fits: two solvers (GPU Levenberg-Marquardt, MINPACK) at one minimum
    for key in ("sigma_lsq", "gamma2_lsq"):
        assert np.allclose(res[key], ref[key], rtol=1e-6, atol=1e-12, equal_nan=True), (key, res[key], ref[key])
    assert np.allclose(res["dF_gauss_lsq"], ref["dF_gauss_lsq"], rtol=1e-6, atol=1e-6, equal_nan=True)
    if int(prob.get("w_half_bins", 0)) > 0:
        assert np.max(np.abs(res["work_hist"] - ref["work_hist"])) < 1e-12
        for key in ("dF_je_hist", "dF_je_hist_mid", "dF_je_hist_literal"):
            assert np.allclose(res[key], ref[key], rtol=1e-9, atol=1e-8, equal_nan=True), key
        assert np.array_equal(res["q_bins"], ref["q_bins"])
        assert np.allclose(res["sigma_w"], ref["sigma_w"], rtol=1e-9, atol=1e-12)
        assert np.allclose(res["dF_je_var_paper"], ref["dF_je_var_paper"], rtol=1e-8, atol=1e-14)
        assert np.allclose(res["work_lost"], ref["work_lost"], atol=1e-12)
        assert np.max(np.abs(res["work_hist_rev"] - ref["work_hist_rev"])) < 1e-12
        for key in ("dF_rev_hist", "dF_crooks"):
            assert np.allclose(res[key], ref[key], rtol=1e-9, atol=1e-8, equal_nan=True), key
        assert np.allclose(res["crooks_ovl"], ref["crooks_ovl"], rtol=0, atol=1e-12)
    else:
        for key in ("dF_rev_hist", "crooks_ovl", "dF_crooks"):
            assert np.all(np.isnan(res[key])), key
    if prob.get("free_ensemble", False):
        on, ron = res["turn_on"], ref["turn_on"]
        for key in ("free_n", "free_blown", "free_under", "free_over"):
            assert on[key] == ron[key], key
        for key in ("eq5_first", "eq6_first", "eq5_last", "eq6_last", "eq10_log", "lower_first", "upper_first",
                    "lower_last", "upper_last", "free_mean", "free_std"):
            assert abs(on[key] - ron[key]) < prof_tol * (1 + abs(ron[key])), (key, on[key], ron[key])
        for key in ("eq5_first_se", "eq6_first_se", "eq5_last_se", "eq6_last_se", "eq10_log_se"):
            assert np.isclose(on[key], ron[key], rtol=1e-7, atol=1e-12, equal_nan=True), key
        assert np.max(np.abs(res["G"] - ref["G"])) < prof_tol * (1 + np.max(np.abs(ref["G"])))
        assert np.allclose(res["G_se"], ref["G_se"], rtol=1e-7, atol=1e-12, equal_nan=True)
        assert np.array_equal(res["xi_hist_free"].astype(np.int64), ref["xi_hist_free"])
    else:
        assert all(np.isnan(v) for v in res["turn_on"].values())
        assert np.all(np.isnan(res["G"])) and not np.any(res["xi_hist_free"])


RUN_CASES = [
    ("1d", dict(n_replicas=300, n_steps=3000, n_windows=21), None),
    ("1d-em", dict(n_replicas=70, n_steps=2000, n_windows=6), {"integrator_1d": 1}),
    ("1d-pull", dict(n_replicas=40, n_steps=2000, n_windows=6), {"n_pull": 500, "n_equil": 500}),
    ("chain10", 10, dict(n_replicas=70, n_steps=600, n_windows=5)),
    ("chain32", 32, dict(n_replicas=70, n_steps=400, n_windows=4)),
    ("chain37", 37, dict(n_replicas=20, n_steps=300, n_windows=4)),
    ("chain100", 100, dict(n_replicas=20, n_steps=300, n_windows=3)),
    ("chain256-pull", 256, dict(n_replicas=5, n_steps=200, n_windows=3)),
]


@pytest.mark.parametrize("case", RUN_CASES, ids=[c[0] for c in RUN_CASES])
def test_run_parity_fp64(case):
    name = case[0]
    _say(f"case run {name}")
    if name.startswith("1d"):
        prob = ppp_inputs.config_1d(precision="fp64", **case[1])
        if case[2]:
            prob.update(case[2])
        prob["w_half_bins"] = 3000
    else:
        prob = ppp_inputs.config_chain_small(case[1], precision="fp64", **case[2])
        prob["w_half_bins"] = 3000
        prob["w_bin"] = 0.05
        if name.endswith("pull"):
            prob["n_pull"] = 100
            prob["n_equil"] = 100
    res, tim = ppp.run(prob)
    xi, kept, _ = oracle.run(prob)
    ref = estimators.estimate(prob, xi, kept)
    _compare_runs(prob, res, ref)


def test_run_parity_fp64_1d_full_size():
    """The 1-D double-well workload at its full size and as the bench runs it
    (21 windows x 256 replicas x 20000 LM steps, fp64, App. C over 2M+1 = 30001
    work bins), element by element against the oracle.  Every window's restrained
    potential is strictly convex (U'' = 60x^2 - 20 + k = 60x^2 + 30 at k = 50), so
    a replica's two fp64 trajectories stay within rounding of each other for the
    whole run and every sample falls in the same bin."""
    prob = ppp_inputs.config_1d()
    _say("case run 1d-full: 21 windows x 256 replicas x 20000 steps, fp64")
    res, tim = ppp.run(prob)
    xi, kept, _ = oracle.run(prob)
    ref = estimators.estimate(prob, xi, kept)
    _compare_runs(prob, res, ref)


def _edge_case(name):
    if name == "smallest":          # N = 2, two windows, one replica, one histogram bin, no App. C
        p = ppp_inputs.config_chain_small(2, n_replicas=1, n_steps=500, n_windows=2, precision="fp64")
        p.update({"xi_nbins": 1, "xi_min": 0.0, "xi_bin": 10.0, "w_half_bins": 0, "n_blocks": 1})
    elif name == "decreasing":      # pulling towards smaller lambda
        p = ppp_inputs.config_chain_small(3, n_replicas=40, n_steps=800, n_windows=5, precision="fp64")
        p["lambda"] = p["lambda"][::-1]
        p["w_half_bins"] = 2000
        p["w_bin"] = 0.05
    elif name == "every-step":      # sample every step from the first one
        p = ppp_inputs.config_1d(n_replicas=50, n_steps=600, n_windows=5)
        p.update({"n_equil": 0, "sample_every": 1, "w_half_bins": 2000})
    elif name == "narrow-histogram":  # most samples fall outside the histogram
        p = ppp_inputs.config_chain_small(10, n_replicas=30, n_steps=400, n_windows=4, precision="fp64")
        lo = p["lambda"][1]
        p.update({"xi_min": lo, "xi_bin": 0.01, "xi_nbins": 50, "w_half_bins": 1000, "w_bin": 0.05})
    else:
        raise ValueError(name)
    return p


@pytest.mark.parametrize("name", ["smallest", "decreasing", "every-step", "narrow-histogram"])
def test_edge_case_parity_fp64(name):
    _say(f"case edge {name}")
    prob = _edge_case(name)
    res, _ = ppp.run(prob)
    xi, kept, _ = oracle.run(prob)
    ref = estimators.estimate(prob, xi, kept)
    _compare_runs(prob, res, ref)
    if name == "narrow-histogram":
        assert res["xi_under_over"].sum() > 0


def test_run_without_samples():
    """Too few steps for any sample: counts are zero and every estimate is
    non-finite, on both sides."""
    _say("case no samples")
    prob = ppp_inputs.config_chain_small(4, n_replicas=8, n_steps=50, n_windows=3, precision="fp64")
    prob.update({"n_equil": 45, "sample_every": 10})
    res, _ = ppp.run(prob)
    xi, kept, _ = oracle.run(prob)
    ref = estimators.estimate(prob, xi, kept)
    assert np.all(res["n_samples"] == 0) and np.all(ref["n_samples"] == 0)
    assert np.all(res["xi_hist"] == 0)
    for key in ("dF_je", "dF_fluct", "dF_gauss"):
        assert not np.any(np.isfinite(res[key][1:])) and not np.any(np.isfinite(ref[key][1:])), key


def test_paper_scale_work_distributions_fp64():
    """App. C at the paper's resolution: x bins of 0.001 over [0, 50] (K = 50000,
    beyond the LDS histogram, so samples go straight to memory) and work bins
    of 0.01 over +-450 (2M+1 = 90001), both work-distribution chains and the
    free ensemble's histogram, against the oracle."""
    _say("case paper-scale App. C")
    prob = ppp_inputs.config_chain_small(10, n_replicas=70, n_steps=600, n_windows=5, precision="fp64")
    prob.update({"xi_min": 0.0, "xi_bin": 0.001, "xi_nbins": 50000, "w_bin": 0.01, "w_half_bins": 45000,
                 "free_ensemble": True})
    res, tim = ppp.run(prob)
    xi, kept, _ = oracle.run(prob)
    ref = estimators.estimate(prob, xi, kept)
    _compare_runs(prob, res, ref)
    _say(f"  appc {tim['appc_ms']:.3f} ms, q_bins {res['q_bins']}")
    assert res["work_hist"].shape == (5, 90001) and np.all(res["q_bins"][1:] > 100)


def _free_case(name):
    if name == "1d-harmonic":       # closed form exists; lambda range not symmetric about 0
        p = ppp_inputs.config_harmonic_1d(kappa=4.0, k=2.0, n_replicas=70, n_steps=2000)
        p["lambda"] = list(np.linspace(-1.0, 0.4, 8))
        p["w_half_bins"] = 0
    elif name == "1d-double-well":  # with App. C
        p = ppp_inputs.config_1d(n_replicas=50, n_steps=2000, n_windows=6)
        p.update({"k": 20.0, "w_half_bins": 2000})
    elif name == "chain10":
        p = ppp_inputs.config_chain_small(10, n_replicas=70, n_steps=600, n_windows=5, precision="fp64")
        p.update({"w_half_bins": 3000, "w_bin": 0.05})
    elif name == "chain32-pull":    # items span windows, the last one into the free ensemble
        p = ppp_inputs.config_chain_small(32, n_replicas=21, n_steps=400, n_windows=3, precision="fp64")
        p.update({"w_half_bins": 0, "n_pull": 100, "n_equil": 100})
    else:
        raise ValueError(name)
    p["free_ensemble"] = True
    return p


@pytest.mark.parametrize("name", ["1d-harmonic", "1d-double-well", "chain10", "chain32-pull"])
def test_free_ensemble_parity_fp64(name):
    """Turn-on free energies (Eqs. 5-7, 10, 15) from the unrestrained ensemble run
    as one more window: every output against the oracle, the per-window profiles
    unchanged by it."""
    _say(f"case free ensemble {name}")
    prob = _free_case(name)
    res, tim = ppp.run(prob)
    xi, kept, _ = oracle.run(prob)
    ref = estimators.estimate(prob, xi, kept)
    _compare_runs(prob, res, ref)
    s, R = len(prob["lambda"]), prob["n_replicas"]
    assert tim["replica_steps"] == (s + 1) * R * prob["n_steps"]
    plain = dict(prob, free_ensemble=False)
    res0, _ = ppp.run(plain)
    for key in ("dF_je", "dF_fluct", "dF_je_se", "xi_mean"):
        assert np.array_equal(res0[key], res[key], equal_nan=True), key
    assert np.array_equal(res0["xi_hist"], res["xi_hist"])


SEQ_CASES = [
    ("1d", None, dict(n_replicas=70, n_steps=800, n_windows=6)),
    ("1d-pull", None, dict(n_replicas=40, n_steps=600, n_windows=4)),
    ("chain10", 10, dict(n_replicas=70, n_steps=300, n_windows=4)),
    ("chain37", 37, dict(n_replicas=20, n_steps=200, n_windows=3)),
    ("chain100", 100, dict(n_replicas=12, n_steps=150, n_windows=3)),
]


@pytest.mark.parametrize("case", SEQ_CASES, ids=[c[0] for c in SEQ_CASES])
def test_sequential_run_parity_fp64(case):
    """Sequential pulling protocol (each replica runs the windows one after
    another) against the oracle, element by element."""
    name, n_beads, kw = case
    _say(f"case sequential {name}")
    if n_beads is None:
        prob = ppp_inputs.config_1d(precision="fp64", **kw)
        if name.endswith("pull"):
            prob["n_pull"] = 200
            prob["n_equil"] = 200
    else:
        prob = ppp_inputs.config_chain_small(n_beads, precision="fp64", **kw)
        prob["w_bin"] = 0.05
    prob["w_half_bins"] = 2000
    prob["sequential"] = True
    res, tim = ppp.run(prob)
    assert tim["replica_steps"] == prob["n_replicas"] * len(prob["lambda"]) * prob["n_steps"]
    xi, kept, _ = oracle.run(prob)
    ref = estimators.estimate(prob, xi, kept)
    _compare_runs(prob, res, ref)


def test_sequential_uneven_chunks_and_frozen_replicas():
    _say("case sequential chunks")
    prob = ppp_inputs.config_chain_small(10, n_replicas=30, n_steps=90, n_windows=4, precision="fp64")
    prob["sequential"] = True
    full, _ = ppp.run(prob)
    h = ppp.ppp_create(prob)
    try:
        ws = ppp.workspace(h)
        ppp.ppp_begin(h, ws)
        for n in [7, 83, 1, 90, 13, 45, 2]:          # stops inside windows and on their boundaries
            ppp.ppp_advance(h, n)
        ppp.ppp_finalize(h)                          # the last window never entered: empty records
        part = ppp.ppp_get_result(h, prob)
        assert ppp.ppp_steps_done(h) == 241
        ppp.ppp_begin(h, ws)
        ppp.ppp_advance(h, 10 ** 9)
        ppp.ppp_finalize(h)
        again = ppp.ppp_get_result(h, prob)
    finally:
        ppp.ppp_destroy(h)
    for key in ("dF_je", "xi_mean", "xi_hist", "n_samples"):
        assert np.array_equal(full[key], again[key]), key
    # 241 steps: windows 1 and 2 complete, window 3 up to step 61 of 90, window 4 empty
    assert np.array_equal(part["n_samples"][:2], full["n_samples"][:2])
    assert 0 < part["n_samples"][2] < full["n_samples"][2] and part["n_samples"][3] == 0
    # a replica that blows up stays frozen in the later windows
    init = ppp_inputs.random_chain_coords(10, 1, seed=4)[0]
    init[5, 1] = np.nan
    prob2 = dict(prob, init_coords=init.ravel().tolist())
    res, _ = ppp.run(prob2)
    assert np.all(res["n_blown_up"] == prob["n_replicas"]) and np.all(res["n_samples"] == 0)


def test_checkpoint_resume_is_bit_identical():
    _say("case checkpoint")
    prob = ppp_inputs.config_chain_small(13, n_replicas=40, n_steps=800, n_windows=4, precision="fp64")
    h = ppp.ppp_create(prob)
    try:
        ws = ppp.workspace(h)
        ppp.ppp_run(h, ws)
        full = ppp.ppp_get_result(h, prob)
        ppp.ppp_begin(h, ws)
        ppp.ppp_advance(h, 333)
        blob = ppp.ppp_checkpoint(h)
        assert ppp.ppp_steps_done(h) == 333
    finally:
        ppp.ppp_destroy(h)
    h2 = ppp.ppp_create(prob)
    try:
        ws2 = ppp.workspace(h2)
        ppp.ppp_restore(h2, ws2, blob)
        ppp.ppp_advance(h2, 10 ** 9)
        ppp.ppp_finalize(h2)
        part = ppp.ppp_get_result(h2, prob)
    finally:
        ppp.ppp_destroy(h2)
    for key in ("dF_je", "dF_fluct", "xi_mean", "xi_hist", "n_samples"):
        assert np.array_equal(full[key], part[key]), key


def test_advancing_in_uneven_chunks_matches_one_run():
    """A launch carries positions and velocities over and recomputes the forces
    from them; advances of 1 to 13 steps must give the single run's results
    exactly, so those recomputed forces have to round as the carried ones did."""
    _say("case uneven chunks")
    for precision in ("fp32", "fp64"):
        prob = ppp_inputs.config_chain_small(10, n_replicas=30, n_steps=240, n_windows=3, precision=precision)
        full, _ = ppp.run(prob)
        h = ppp.ppp_create(prob)
        try:
            ws = ppp.workspace(h)
            ppp.ppp_begin(h, ws)
            for n in [1, 2, 3, 5, 6, 7, 9, 13] * 4:
                ppp.ppp_advance(h, n)
            ppp.ppp_advance(h, 10 ** 9)
            ppp.ppp_finalize(h)
            part = ppp.ppp_get_result(h, prob)
        finally:
            ppp.ppp_destroy(h)
        for key in ("dF_je", "dF_fluct", "xi_mean", "xi_std", "xi_hist", "n_samples"):
            assert np.array_equal(full[key], part[key]), (precision, key)


def test_frozen_replicas_are_counted():
    _say("case blowup")
    prob = ppp_inputs.config_chain_small(10, n_replicas=16, n_steps=100, n_windows=3, precision="fp32")
    init = ppp_inputs.random_chain_coords(10, 1, seed=4)[0]
    init[5, 1] = np.nan
    prob["init_coords"] = init.ravel().tolist()
    res, _ = ppp.run(prob)
    assert res["status"] == ppp.PPP_E_NUMERICAL
    assert np.all(res["n_blown_up"] == 16) and np.all(res["n_samples"] == 0)


def test_fp32_chain_statistics_match_oracle():
    """fp32 forces with fp64 accumulation: final dF within 3 combined standard errors of the fp64 oracle."""
    _say("case fp32 statistics chain10")
    prob = ppp_inputs.config_chain10(n_replicas=128, n_steps=6000)
    prob["n_blocks"] = 16
    res, _ = ppp.run(prob)
    p64 = dict(prob, precision="fp64")
    xi, kept, _ = oracle.run(p64)
    ref = estimators.estimate(p64, xi, kept, with_appc=False)
    for key in ("dF_je", "dF_fluct", "dF_gauss"):
        se = np.sqrt(res[key + "_se"][-1] ** 2 + ref[key + "_se"][-1] ** 2)
        assert abs(res[key][-1] - ref[key][-1]) < 3.0 * se, (key, res[key][-1], ref[key][-1], se)


FP32_SLICES = [
    # (name, problem, estimators asserted): the workloads' own step counts, fewer replicas
    ("chain10", lambda: ppp_inputs.config_chain10(n_replicas=64), ("dF_je", "dF_fluct", "dF_gauss", "dF_com")),
    # uniform windows up to 5.7 sigma apart: JE rests on rare samples there and its
    # jackknife error is large, but it is still asserted at 3 combined SE
    ("chain32", lambda: ppp_inputs.config_chain32(n_replicas=16), ("dF_je", "dF_fluct", "dF_gauss", "dF_com")),
]


@pytest.mark.parametrize("case", FP32_SLICES, ids=[c[0] for c in FP32_SLICES])
def test_fp32_error_vs_fp64_oracle(case):
    """Precision split: fp32 forces and integration with fp64 work accumulation
    against the all-fp64 oracle on the same inputs and noise streams; the error
    of every dF at the last window is printed and checked against 3 combined
    jackknife standard errors."""
    name, make, asserted = case
    _say(f"case fp32 vs fp64 oracle {name}")
    prob = make()
    prob["n_blocks"] = 16
    res, _ = ppp.run(prob)
    p64 = dict(prob, precision="fp64")
    xi, kept, _ = oracle.run(p64)
    ref = estimators.estimate(p64, xi, kept, with_appc=False)
    line = []
    for key in ("dF_je", "dF_fluct", "dF_gauss", "dF_com"):
        err = res[key][-1] - ref[key][-1]
        se = np.sqrt(res[key + "_se"][-1] ** 2 + ref[key + "_se"][-1] ** 2)
        line.append(f"{key} gpu {res[key][-1]:.4f} oracle {ref[key][-1]:.4f} err {err:+.4f} (combined se {se:.4f})")
        if key in asserted:
            assert abs(err) < 3.0 * se, line[-1]
    _say(f"fp32 error {name}: " + "; ".join(line))


def _window_mean_z(res, xi, kept, R):
    """z of the fp32 window means against the fp64 oracle's: the oracle's replicas
    give the standard error of one run's window mean (replica means are
    independent); the two runs have the same spread, so the difference has sqrt(2)
    times that error."""
    s = len(res["xi_mean"])
    z = np.zeros(s)
    for w in range(s):
        rows = xi[w * R:(w + 1) * R]
        n = kept[w * R:(w + 1) * R]
        m = np.array([rows[r, :n[r]].mean() for r in range(R) if n[r] > 0])
        se = np.sqrt(2.0) * m.std(ddof=1) / np.sqrt(len(m))
        z[w] = (res["xi_mean"][w] - rows[~np.isnan(rows)].mean()) / se
    return z


@pytest.mark.slow
def test_fp32_error_vs_fp64_oracle_chain256():
    """Precision split on the 256-bead workload: fp32 forces and integration with
    fp64 work against the all-fp64 oracle on every one of its 41 windows, 16
    replicas each, 3000 steps with the pull from the helix over the first 2000
    (the full run pulls over 10000 of its 200000; a faster pull than this
    compresses the chain into Lennard-Jones overlaps in the low windows).  The
    windows do not relax in 1000 steps, which both sides share: the comparison
    is of the same non-equilibrium protocol.  Eq. 14 and Eq. 13 at the last
    window within 3 combined jackknife SE; the 41 window means through their z
    values (mean z^2 near 1; the largest of 41 below 4.5); the JE error printed,
    not asserted: these windows lie about 20 sigma apart, where JE rests on the
    rarest samples (Sec. IV B)."""
    _say("case fp32 vs fp64 oracle chain256 (41 windows x 16 replicas x 3000 steps)")
    prob = ppp_inputs.config_chain256(n_replicas=16, n_steps=3000)
    prob.update({"n_pull": 2000, "n_equil": 2000, "n_blocks": 8})
    res, _ = ppp.run(prob)
    p64 = dict(prob, precision="fp64")
    xi, kept, _ = oracle.run(p64)
    ref = estimators.estimate(p64, xi, kept, with_appc=False)
    assert int(res["n_blown_up"].sum()) == 0 and int(ref["n_blown_up"].sum()) == 0
    line = []
    for key in ("dF_je", "dF_fluct", "dF_gauss", "dF_com"):
        err = res[key][-1] - ref[key][-1]
        se = np.sqrt(res[key + "_se"][-1] ** 2 + ref[key + "_se"][-1] ** 2)
        line.append(f"{key} gpu {res[key][-1]:.3f} oracle {ref[key][-1]:.3f} err {err:+.3f} (combined se {se:.3f})")
        if key in ("dF_fluct", "dF_gauss"):
            assert abs(err) < 3.0 * se, line[-1]
    z = _window_mean_z(res, xi, kept, 16)
    _say("fp32 error chain256: " + "; ".join(line))
    _say(f"  window means: mean z^2 {np.mean(z ** 2):.2f}, max |z| {np.max(np.abs(z)):.2f}; "
         f"max dlambda/sigma {np.max(res['dlambda_over_sigma']):.1f}")
    assert np.mean(z ** 2) < 2.0 and np.max(np.abs(z)) < 4.5


# four chains of the uneven batch, one per kernel shape of its length class
C2_SLICE = (5, 9, 61, 11)


@pytest.mark.slow
def test_fp32_batch_error_vs_fp64_oracle():
    """Precision split on the uneven batch: four of its chains (8, 23, 52 and 128
    beads, one per kernel shape the batch uses for them) with their own windows,
    32 replicas each and a shortened schedule (3000 steps, the pull and the
    equilibration over the first 1000), run in fp32 as one batched graph, against
    the fp64 oracle on each problem.  Eq. 14 and Eq. 13 within 3 combined SE;
    JE asserted where adjacent windows lie within 3 sigma, printed elsewhere."""
    inst = ppp_inputs.batched_instances()
    probs = []
    for i in C2_SLICE:
        p = dict(inst[i])
        p.update({"n_replicas": 32, "n_steps": 3000, "n_equil": 1000, "n_pull": 1000, "n_blocks": 16,
                  "w_half_bins": 0})
        probs.append(p)
    _say("case fp32 batch vs fp64 oracle, chains " + ", ".join(f"N={p['n_beads']}" for p in probs))
    h = ppp.ppp_batch_create(probs)
    try:
        ws = ppp.workspace(h)
        ppp.ppp_run(h, ws)
        torch.cuda.synchronize()
        got = [ppp.ppp_batch_get_result(h, p, i) for i, p in enumerate(probs)]
    finally:
        ppp.ppp_destroy(h)
    for p, res in zip(probs, got):
        p64 = dict(p, precision="fp64")
        xi, kept, _ = oracle.run(p64)
        ref = estimators.estimate(p64, xi, kept, with_appc=False)
        assert int(res["n_blown_up"].sum()) == 0 and int(ref["n_blown_up"].sum()) == 0
        dls = float(np.max(ref["dlambda_over_sigma"]))
        asserted = ("dF_fluct", "dF_gauss") + (("dF_je", "dF_com") if dls <= 3.0 else ())
        line = []
        for key in ("dF_je", "dF_fluct", "dF_gauss", "dF_com"):
            err = res[key][-1] - ref[key][-1]
            se = np.sqrt(res[key + "_se"][-1] ** 2 + ref[key + "_se"][-1] ** 2)
            line.append(f"{key} err {err:+.3f} (se {se:.3f})")
            if key in asserted:
                assert abs(err) < 3.0 * se, (p["name"], line[-1])
        _say(f"fp32 error batch {p['name']} N={p['n_beads']} max dl/sigma {dls:.1f}: " + "; ".join(line))


def _shapes():
    from paper_1105_4840_amd import build
    return build.shapes()


@pytest.mark.parametrize("shape", _shapes(), ids=lambda s: f"{s[0]}x{s[1]}")
def test_every_kernel_shape_fp64_trajectory_and_forces(shape, tmp_path, monkeypatch):
    """Each compiled (lanes x beads-per-lane) shape, forced through the shape table:
    fp64 100-step trajectory within 1e-10 and fp32 forces within 1e-5 of the oracle."""
    G, B = shape
    n = max(2, G * B - (B // 2))          # leaves some padding beads in the last lane
    _say(f"case shape {G}x{B} N={n}")
    table = tmp_path / "tune.txt"
    table.write_text(f"{n} 1 {G} {B}\n{n} 0 {G} {B}\n")
    monkeypatch.setenv("PPP_TUNE_TABLE", str(table))
    prob = ppp_inputs.config_chain_small(n, n_replicas=6, n_steps=100, n_windows=3, precision="fp64")
    h = ppp.ppp_create(prob)
    try:
        ws = ppp.workspace(h)
        tr = ppp.ppp_trajectory(h, ws, 2, 5, 100, 3 * n).cpu().numpy()
    finally:
        ppp.ppp_destroy(h)
    ref = oracle.trajectory(prob, 2, 5, 100)
    assert np.max(np.abs(tr - ref)) < 1e-10, np.max(np.abs(tr - ref))
    p32 = dict(prob, precision="fp32")
    conf = ppp_inputs.random_chain_coords(n, 3, seed=G * 100 + B)
    h = ppp.ppp_create(p32)
    try:
        ws = ppp.workspace(h)
        x = torch.tensor(conf.reshape(len(conf), -1), dtype=torch.float64, device="cuda")
        f, e = ppp.ppp_eval_forces(h, ws, x, 0.4 * n)
        f = f.cpu().numpy().reshape(len(conf), -1, 3)
    finally:
        ppp.ppp_destroy(h)
    for c in range(len(conf)):
        xc = conf[c].astype(np.float32).astype(np.float64)
        _, _, fr = oracle.chain_forces(p32, xc, 0.4 * n)
        assert np.linalg.norm(f[c, 1:] - fr[1:]) <= 1e-5 * np.linalg.norm(fr[1:])


@pytest.mark.parametrize("shape", _shapes(), ids=lambda s: f"{s[0]}x{s[1]}")
def test_every_kernel_shape_resumes_bit_exactly(shape, tmp_path, monkeypatch):
    """The uneven-chunk check for every compiled shape, forced through the shape
    table, in both precisions: the forces each advance recomputes from the stored
    state must round as the ones the uninterrupted run carried, whatever the
    compiler does with the inlined force code of that shape."""
    G, B = shape
    n = max(2, G * B - (B // 2))
    table = tmp_path / "tune.txt"
    table.write_text(f"{n} 1 {G} {B}\n{n} 0 {G} {B}\n")
    monkeypatch.setenv("PPP_TUNE_TABLE", str(table))
    for precision in ("fp32", "fp64"):
        _say(f"case resume shape {G}x{B} N={n} {precision}")
        prob = ppp_inputs.config_chain_small(n, n_replicas=6, n_steps=120, n_windows=3, precision=precision)
        full, _ = ppp.run(prob)
        h = ppp.ppp_create(prob)
        try:
            ws = ppp.workspace(h)
            ppp.ppp_begin(h, ws)
            for k in [1, 2, 3, 5, 7, 13] * 3:
                ppp.ppp_advance(h, k)
            ppp.ppp_advance(h, 10 ** 9)
            ppp.ppp_finalize(h)
            part = ppp.ppp_get_result(h, prob)
        finally:
            ppp.ppp_destroy(h)
        for key in ("dF_je", "xi_mean", "xi_std", "xi_hist", "n_samples"):
            assert np.array_equal(full[key], part[key], equal_nan=True), (precision, key)



def test_valu_probe_computes_its_chains():
    """The issue-rate probe does the arithmetic it is credited with: every thread's
    output is the sum of its 8 FMA chains, recomputed here in fp64 from the fp32
    start values (fp32 rounding each step keeps it within 1e-5 relative), with
    its operands in scalar registers and, bit for bit the same, in vector ones."""
    _say("case valu probe")
    n_blocks, iters, b, c = 3, 50, 0.999, 1e-3
    out = ppp.ppp_probe_valu(n_blocks, iters, b=b, c=c).cpu().numpy().astype(np.float64)
    out_v = ppp.ppp_probe_valu(n_blocks, iters, b=b, c=c, vgpr_operands=True).cpu().numpy().astype(np.float64)
    assert np.array_equal(out, out_v)
    i = np.arange(n_blocks * 256)
    want = np.zeros_like(out)
    b32, c32 = float(np.float32(b)), float(np.float32(c))
    for k in range(8):
        a = np.float32(((i + k) & 1023) * np.float32(1e-6)).astype(np.float64)
        for _ in range(iters):
            a = a * b32 + c32
        want += a
    assert np.allclose(out, want, rtol=1e-5, atol=0)
    with pytest.raises(ppp.PppError):
        ppp.ppp_probe_valu(0, 10)
