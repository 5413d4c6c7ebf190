"""The allocation-free entry point ppp_run_static (needs an MI355X): its results
equal those of ppp_run with a caller workspace, element for element, on two
calls in a row, the second with a smaller problem (the static workspace keeps
the first call's contents, which the run must not read); problems too large
for the static workspace and batched handles are refused before device work."""
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


def _static_run(prob):
    h = ppp.ppp_create(prob)
    try:
        assert ppp.ppp_workspace_size(h) <= ppp.PPP_STATIC_WORKSPACE_BYTES
        st = ppp.lib().ppp_run_static(h, ppp._stream())
        assert st in (ppp.PPP_OK, ppp.PPP_E_NUMERICAL), ppp.lib().ppp_last_error(h)
        return ppp.ppp_get_result(h, prob)
    finally:
        ppp.ppp_destroy(h)


def _same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    if np.issubdtype(a.dtype, np.floating):
        return np.array_equal(a, b, equal_nan=True)
    return np.array_equal(a, b)


def test_static_workspace_matches_caller_workspace_on_two_calls():
    big = ppp_inputs.config_chain_small(10, n_replicas=70, n_steps=600, n_windows=5, precision="fp64")
    big.update({"w_half_bins": 3000, "w_bin": 0.05})
    small = ppp_inputs.config_1d(n_replicas=40, n_steps=800, n_windows=4, precision="fp64")
    small["w_half_bins"] = 500
    for prob in (big, small):
        _say(f"case static workspace {prob['name']}")
        ref, _ = ppp.run(prob)
        got = _static_run(prob)
        checked = 0
        for key, v in ref.items():
            if isinstance(v, np.ndarray):
                assert _same(v, got[key]), key
                checked += 1
            elif isinstance(v, dict):
                for k2, v2 in v.items():
                    assert _same(v2, got[key][k2]), (key, k2)
        assert checked > 20


def test_static_workspace_refuses_what_does_not_fit():
    _say("case static workspace limits")
    prob = ppp_inputs.config_chain256(n_replicas=64, n_steps=100)
    h = ppp.ppp_create(prob)
    try:
        assert ppp.ppp_workspace_size(h) > ppp.PPP_STATIC_WORKSPACE_BYTES
        assert ppp.lib().ppp_run_static(h, ppp._stream()) == ppp.PPP_E_OUT_OF_MEMORY
        assert b"static workspace" in ppp.lib().ppp_last_error(h)
    finally:
        ppp.ppp_destroy(h)
    hb = ppp.ppp_batch_create(ppp_inputs.batched_instances(2, seed=3))
    try:
        assert ppp.lib().ppp_run_static(hb, ppp._stream()) == ppp.PPP_E_UNSUPPORTED
    finally:
        ppp.ppp_destroy(hb)
