"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, and validates problems before any device work."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1105_4840_amd as ppp
import ppp_inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    """Every function declared in include/*.h."""
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    return sorted(set(re.findall(r"^(?:ppp_status|const char \*)\s*(ppp_\w+)\(", text, flags=re.M)))


def test_header_symbols_exported():
    names = _declared()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", ppp.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (ppp_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = ppp.lib()
    for n in names:
        assert getattr(L, n) is not None
    assert set(ppp.EXPORTED) >= set(names)


def _status(prob):
    p, keep = ppp.make_problem(prob)
    h = ctypes.c_void_p()
    st = ppp.lib().ppp_create(ctypes.byref(p), ctypes.byref(h))
    if st == 0:
        ppp.lib().ppp_destroy(h)
    return st


@pytest.mark.parametrize("mutate", [
    lambda p: p.update(k=0.0),
    lambda p: p.update(kT=-1.0),
    lambda p: p.update(dt=float("nan")),
    lambda p: p.update(n_replicas=0),
    lambda p: p.update(sample_every=0),
    lambda p: p.update(n_equil=p["n_steps"]),
    lambda p: p.update(xi_nbins=0),
    lambda p: p.update(xi_nbins=(1 << 26) + 1),
    lambda p: p.update(xi_nbins=2 ** 31 - 1),
    lambda p: p.update(w_half_bins=50000001),
    lambda p: p.update(xi_bin=0.0),
    lambda p: p.update(w_bin=0.0),
    lambda p: p.update(n_blocks=10 ** 6),
    lambda p: p.update(n_blocks=-1),
    lambda p: p.update(flags=4),
    lambda p: p.update(flags=0x80000001),
    lambda p: p.update(sequential=True, n_steps=2 ** 31, n_equil=0),   # 21 x 2^31 steps per replica
    lambda p: p.update({"lambda": [0.0]}),
    lambda p: p.update({"lambda": [0.0, 1.0, 1.0]}),
    lambda p: p.update({"lambda": [0.0, 1.0, 0.5]}),
    lambda p: p.update({"lambda": [0.0, float("inf")]}),
    lambda p: p.update(n_beads=1),
    lambda p: p.update(n_beads=100000),
    lambda p: p.update(mass=0.0),
    lambda p: p.update(rc_mode=3),
    # the centre would still move while samples are taken (n_equil = 10 here)
    lambda p: p.update(n_pull=11),
])
def test_invalid_chain_problems_rejected(mutate):
    p = ppp_inputs.config_chain10(n_replicas=8, n_steps=100)
    mutate(p)
    assert _status(p) == ppp.PPP_E_INVALID_ARG


def test_invalid_1d_problems_rejected():
    p = ppp_inputs.config_1d(n_replicas=4, n_steps=100)
    p["mobility"] = 0.0
    assert _status(p) == ppp.PPP_E_INVALID_ARG
    p = ppp_inputs.config_1d(n_replicas=4, n_steps=100)
    p["integrator_1d"] = 7
    assert _status(p) == ppp.PPP_E_INVALID_ARG
    p = ppp_inputs.config_1d(n_replicas=4, n_steps=100)
    p["pot_kind"] = 9
    assert _status(p) == ppp.PPP_E_INVALID_ARG


def test_pull_ending_at_the_first_sample_is_accepted():
    p = ppp_inputs.config_chain10(n_replicas=8, n_steps=100)
    p["n_pull"] = p["n_equil"]
    assert _status(p) == 0
    p["n_pull"] = p["n_equil"] + 1
    assert _status(p) == ppp.PPP_E_INVALID_ARG
    assert "n_pull" in ppp.lib().ppp_create_error().decode()


def test_valid_problems_and_workspace_size():
    for p in (ppp_inputs.config_1d(), ppp_inputs.config_chain10(), ppp_inputs.config_chain32(),
              ppp_inputs.config_chain256()):
        h = ppp.ppp_create(p)
        n = ppp.ppp_workspace_size(h)
        assert n > 0 and n % 256 == 0
        ppp.ppp_destroy(h)
    # descending windows are allowed too
    p = ppp_inputs.config_chain10(n_replicas=8, n_steps=100)
    p["lambda"] = p["lambda"][::-1]
    assert _status(p) == 0


def test_sequential_protocol_accepted_where_supported():
    p = ppp_inputs.config_chain10(n_replicas=8, n_steps=100)
    p["sequential"] = True
    assert _status(p) == 0
    h = ppp.ppp_create(p)
    try:
        # trajectories are recorded for the parallel protocol only
        assert ppp.lib().ppp_trajectory(h, None, 0, 0, 0, 10, None, None) in (ppp.PPP_E_UNSUPPORTED, ppp.PPP_E_INVALID_ARG)
    finally:
        ppp.ppp_destroy(h)
    with pytest.raises(ppp.PppError):
        ppp.ppp_batch_create([p, dict(p)])


def test_free_ensemble_accepted_where_supported():
    """The unrestrained ensemble runs with the parallel protocol, batched too; not
    with the sequential protocol nor for window placement."""
    p = ppp_inputs.config_chain10(n_replicas=8, n_steps=100)
    p["free_ensemble"] = True
    assert _status(p) == 0
    assert _status(dict(p, sequential=True)) == ppp.PPP_E_UNSUPPORTED
    q = ppp_inputs.config_1d(n_replicas=8, n_steps=100)
    q["free_ensemble"] = True
    assert _status(q) == 0
    h = ppp.ppp_batch_create([p, dict(p, n_beads=12)])
    assert ppp.ppp_workspace_size(h) > 0
    ppp.ppp_destroy(h)
    # one more window of replicas, records and histogram in the workspace
    h0, h1 = ppp.ppp_create(dict(p, free_ensemble=False)), ppp.ppp_create(p)
    try:
        assert ppp.ppp_workspace_size(h1) > ppp.ppp_workspace_size(h0)
    finally:
        ppp.ppp_destroy(h0); ppp.ppp_destroy(h1)
    pb, keep = ppp.make_problem(p)
    ad = ppp.ppp_adaptive(budget_replica_steps=10 ** 9, initial_windows=5, max_rounds=2, max_windows=16,
                          target_dl_over_sigma=1.0, train_iters=10, lr=1e-3, init_seed=1, explore_replicas=8,
                          explore_steps=100, min_production_steps=100)
    n = ctypes.c_size_t()
    assert ppp.lib().ppp_adaptive_workspace_size(ctypes.byref(pb), ctypes.byref(ad), ctypes.byref(n)) == ppp.PPP_E_UNSUPPORTED


def test_error_strings():
    L = ppp.lib()
    for s in range(7):
        assert L.ppp_status_string(s)
    assert L.ppp_last_error(None) == b""
    p = ppp_inputs.config_chain10(n_replicas=8, n_steps=100)
    p["k"] = -1.0
    with pytest.raises(ppp.PppError) as e:
        ppp.ppp_create(p)
    assert "k must be" in str(e.value)


def test_batch_rejects_1d():
    with pytest.raises(ppp.PppError):
        ppp.ppp_batch_create([ppp_inputs.config_1d(n_replicas=4, n_steps=100)])
    h = ppp.ppp_batch_create(ppp_inputs.batched_instances(6, seed=3))
    assert ppp.ppp_workspace_size(h) > 0
    ppp.ppp_destroy(h)


def test_autotune_rejects_null_path():
    assert ppp.lib().ppp_autotune(None, None, 0, None) == ppp.PPP_E_INVALID_ARG


def test_valu_probe_rejects_bad_arguments_before_any_launch():
    """The issue-rate probe checks its arguments on the host: an unknown operand
    form, no blocks, no steps or a NULL output are refused without a launch."""
    import ctypes
    L = ppp.lib()
    dummy = ctypes.c_void_p(16)   # never dereferenced: every call below is refused first
    assert L.ppp_probe_valu(1, 1, 1.0, 0.0, 7, dummy, None) == ppp.PPP_E_INVALID_ARG
    assert L.ppp_probe_valu(1, 1, 1.0, 0.0, -1, dummy, None) == ppp.PPP_E_INVALID_ARG
    assert L.ppp_probe_valu(0, 1, 1.0, 0.0, ppp.PPP_PROBE_VGPR_OPERANDS, dummy, None) == ppp.PPP_E_INVALID_ARG
    assert L.ppp_probe_valu(1, 0, 1.0, 0.0, ppp.PPP_PROBE_SGPR_OPERANDS, dummy, None) == ppp.PPP_E_INVALID_ARG
    assert L.ppp_probe_valu(1, 1, 1.0, 0.0, ppp.PPP_PROBE_SGPR_OPERANDS, None, None) == ppp.PPP_E_INVALID_ARG
