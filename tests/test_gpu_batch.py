"""Batched uneven problems in one persistent, graph-captured launch (needs an MI355X).

Every replica's trajectory and every reduction are independent of how work is
scheduled, so each problem of a batch must reproduce its own single run
exactly (fp32 and fp64), on every replay of the captured graph; fp64 batches
also match the oracle."""
import sys

import numpy as np
import pytest

import oracle
import paper_1105_4840_amd as ppp
import ppp_inputs
from oracle import estimators

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("dF_je", "dF_fluct", "dF_gauss", "dF_je_se", "xi_mean", "xi_std", "n_samples", "xi_hist", "dF_je_hist",
        "work_hist", "overlap_ovl", "kish_frac", "work_hist_rev", "dF_crooks", "sigma_lsq", "dF_gauss_lsq",
        "dF_je_hist_literal")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _small_batch(n, seed, precision, steps_scale=0.02, rep_cap=64):
    """Uneven chains, windows, replicas and steps as in the batched workload, with the
    windows bracketing the start state so no trajectory explodes (an exploding
    trajectory amplifies any rounding difference without bound)."""
    probs = ppp_inputs.batched_instances(n, seed=seed)
    for p in probs:
        N = p["n_beads"]
        p["lambda"] = list(np.linspace(0.3 * (N - 1) + 0.5, 0.5 * (N - 1) + 1.5, len(p["lambda"])))
        p["n_steps"] = max(200, int(p["n_steps"] * steps_scale))
        p["n_equil"] = p["n_steps"] // 10
        p["n_pull"] = 0
        p["n_replicas"] = min(p["n_replicas"], rep_cap)
        p["precision"] = precision
        p["w_half_bins"] = 2000
        p["w_bin"] = 0.05
    return probs


def _equal(a, b, key):
    if np.issubdtype(np.asarray(a).dtype, np.floating):
        return np.array_equal(a, b, equal_nan=True)
    return np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_matches_single_runs_on_every_replay(precision):
    probs = _small_batch(7, seed=5, precision=precision)
    _say(f"case batch {precision}: N = {[p['n_beads'] for p in probs]}")
    singles = [ppp.run(p)[0] for p in probs]
    h = ppp.ppp_batch_create(probs)
    try:
        ws = ppp.workspace(h)
        for replay in range(3):
            ppp.ppp_run(h, ws)
            torch.cuda.synchronize()
            # eager work between replays
            x = torch.randn(1 << 20, device="cuda"); (x * 2).sum().item()
            for i, p in enumerate(probs):
                r = ppp.ppp_batch_get_result(h, p, i)
                for key in KEYS:
                    assert _equal(r[key], singles[i][key], key), (replay, i, key)
    finally:
        ppp.ppp_destroy(h)


def test_batch_with_free_ensembles_matches_single_runs():
    """Problems that also sample the unrestrained ensemble (one more window of
    replicas each) mixed with plain ones in one batch: every output, the
    turn-on values included, equals the problem's own single run."""
    probs = _small_batch(6, seed=13, precision="fp32")
    for i, p in enumerate(probs):
        p["free_ensemble"] = i % 2 == 0
    _say(f"case batch free ensembles: N = {[p['n_beads'] for p in probs]}")
    singles = [ppp.run(p)[0] for p in probs]
    h = ppp.ppp_batch_create(probs)
    try:
        ws = ppp.workspace(h)
        for replay in range(2):
            ppp.ppp_run(h, ws)
            torch.cuda.synchronize()
            for i, p in enumerate(probs):
                r = ppp.ppp_batch_get_result(h, p, i)
                for key in KEYS + ("G", "G_se", "xi_hist_free"):
                    assert _equal(r[key], singles[i][key], key), (replay, i, key)
                for key, v in singles[i]["turn_on"].items():
                    assert np.array_equal(r["turn_on"][key], v, equal_nan=True), (replay, i, key)
                assert np.isfinite(r["turn_on"]["eq6_first"]) == p["free_ensemble"]
    finally:
        ppp.ppp_destroy(h)


def test_batch_fp64_matches_oracle():
    probs = _small_batch(3, seed=9, precision="fp64", steps_scale=0.005, rep_cap=12)
    _say(f"case batch oracle: N = {[p['n_beads'] for p in probs]}")
    h = ppp.ppp_batch_create(probs)
    try:
        ws = ppp.workspace(h)
        ppp.ppp_run(h, ws)
        for i, p in enumerate(probs):
            r = ppp.ppp_batch_get_result(h, p, i)
            xi, kept, _ = oracle.run(p)
            ref = estimators.estimate(p, xi, kept)
            assert np.array_equal(r["n_samples"], ref["n_samples"])
            assert np.array_equal(r["xi_hist"].astype(np.int64), ref["xi_hist"])
            assert np.allclose(r["xi_mean"], ref["xi_mean"], rtol=1e-10, atol=1e-12)
            assert np.max(np.abs(r["dF_je"] - ref["dF_je"])) < 1e-8 * (1 + np.max(np.abs(ref["dF_je"])))
    finally:
        ppp.ppp_destroy(h)


def test_autotune_table_and_tuned_batch(tmp_path, monkeypatch):
    _say("case autotune")
    path = tmp_path / "tune.txt"
    ws = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    st = ppp.lib().ppp_autotune(str(path).encode(), ppp._ptr(ws), ws.numel(), ppp._stream())
    assert st == ppp.PPP_OK, ppp.lib().ppp_status_string(st)
    rows = [l.split() for l in path.read_text().splitlines() if l and not l.startswith("#")]
    assert len(rows) >= 20
    for r in rows:
        nmax, prec, G, B = (int(x) for x in r[:4])
        assert prec in (0, 1) and G * B >= nmax and 1 <= G <= 64
    del ws
    monkeypatch.setenv("PPP_TUNE_TABLE", str(path))
    probs = _small_batch(4, seed=11, precision="fp32")
    singles = [ppp.run(p)[0] for p in probs]
    h = ppp.ppp_batch_create(probs, str(path))
    try:
        w = ppp.workspace(h)
        ppp.ppp_run(h, w)
        for i, p in enumerate(probs):
            r = ppp.ppp_batch_get_result(h, p, i)
            for key in KEYS:
                assert _equal(r[key], singles[i][key], key), (i, key)
    finally:
        ppp.ppp_destroy(h)
