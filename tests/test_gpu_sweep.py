"""Relaxation-time and stiffness sweep on the 10-bead chain (needs an MI355X):
the claims of the paper's tau and k studies (Sec. IV C-D, Figs. 5-6) checked on
the synthetic chain, all problems in one batched graph launch.

- tau: windows that have not relaxed bias the estimates, JE worst of all; once
  the windows relax (40000 steps and twice that here; a tenth of each run is
  equilibration), a longer relaxation no longer moves dF^JE beyond its error.
- k at fixed windows: a stiffer restraint narrows rho_i, so dlambda/sigma grows
  and the adjacent overlap and the Kish effective-sample fraction of the step
  work fall (the overlap criterion of Sec. IV B).
"""
import sys

import numpy as np
import pytest

import paper_1105_4840_amd as ppp
import ppp_inputs

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


TAUS = (500, 40000, 80000)
KS = (5.0, 20.0, 200.0)


@pytest.fixture(scope="module")
def sweep():
    probs, labels = [], []
    for i, t in enumerate(TAUS):
        probs.append(ppp_inputs.config_chain10(n_replicas=4096, n_steps=t, seed=31 + i))
        labels.append(("tau", t))
    for i, k in enumerate(KS):
        p = ppp_inputs.config_chain10(n_replicas=2048, n_steps=20000, seed=41 + i)
        p["k"] = k
        probs.append(p)
        labels.append(("k", k))
    _say("case sweep: one batched graph of " + ", ".join(f"{a}={b}" for a, b in labels))
    h = ppp.ppp_batch_create(probs)
    try:
        ws = ppp.workspace(h)
        ppp.ppp_run(h, ws)
        torch.cuda.synchronize()
        out = {lab: ppp.ppp_batch_get_result(h, p, i) for i, (p, lab) in enumerate(zip(probs, labels))}
    finally:
        ppp.ppp_destroy(h)
    for lab, r in out.items():
        _say(f"  {lab}: dF_je {r['dF_je'][-1]:+.4f} +- {r['dF_je_se'][-1]:.4f}, dF_fluct {r['dF_fluct'][-1]:+.4f}, "
             f"max dl/sigma {np.max(r['dlambda_over_sigma']):.2f}, min OVL {np.min(r['overlap_ovl']):.3f}, "
             f"min Kish {np.min(r['kish_frac']):.2e}, frozen {int(r['n_blown_up'].sum())}")
    return out


def test_relaxed_windows_agree_and_unrelaxed_ones_are_biased(sweep):
    a, b, c = sweep[("tau", 80000)], sweep[("tau", 40000)], sweep[("tau", 500)]
    for r in (a, b, c):
        assert int(r["n_blown_up"].sum()) == 0
    se = np.hypot(a["dF_je_se"][-1], b["dF_je_se"][-1])
    assert abs(a["dF_je"][-1] - b["dF_je"][-1]) < 3.0 * se
    se_c = np.hypot(a["dF_je_se"][-1], c["dF_je_se"][-1])
    assert abs(c["dF_je"][-1] - a["dF_je"][-1]) > 10.0 * se_c


def test_stiffer_restraint_loses_overlap(sweep):
    r = [sweep[("k", k)] for k in KS]
    dls = [np.max(x["dlambda_over_sigma"]) for x in r]
    ovl = [np.min(x["overlap_ovl"]) for x in r]
    kish = [np.min(x["kish_frac"]) for x in r]
    assert dls[0] < dls[1] < dls[2]
    assert ovl[0] > ovl[1] > ovl[2]
    assert kish[0] > kish[1] > kish[2]
    # the reach criterion of Sec. IV B holds everywhere at k = 5 and fails somewhere at k = 200
    assert np.all(r[0]["criterion_ok"] == 1)
    assert np.any(r[2]["criterion_ok"] == 0)
    # and the error bar of JE grows with the loss of overlap
    assert r[0]["dF_je_se"][-1] < r[2]["dF_je_se"][-1]
