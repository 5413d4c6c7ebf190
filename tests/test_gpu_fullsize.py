"""Full-size parity in the launch the bench times (needs an MI355X): the
10-bead workload (21 windows x 1024 replicas), the 32-bead one (21 x 4096)
and the 256-bead one (41 x 4096), fp32, advanced by one launch of a few steps over
every replica, as `bench.py` launches them.  The state of sampled replicas is
read from the checkpoint (layout in include/ppp.h) and compared with the fp64
oracle's trajectory of the same replica: the first and last replica of the
grid, both sides of a work item's end and of a window boundary.  The fp32
state starts from fp32-rounded coordinates (the 256-bead helix reaches 100,
where fp32 values are 7.6e-6 apart) and takes fp32 forces (1e-5) and normals
(1e-7) for a few steps of dt = 0.005, so it stays within 1e-4 of the fp64
trajectory (measured: 1.1e-6 and 2.4e-5); a replica read at the wrong place,
run on the wrong noise stream or from the wrong start state would be off by
1e-2 or more (the start velocities alone move a bead 0.025 in 5 steps).
The uneven batch runs whole, in its one graph launch, and sampled problems
are checked against their own single runs bit for bit."""
import sys

import numpy as np
import pytest

import oracle
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


def _run_and_sample(prob, steps, picks):
    h = ppp.ppp_create(prob)
    try:
        ws = ppp.workspace(h)
        ppp.ppp_begin(h, ws)
        ppp.ppp_advance(h, steps)
        ppp.ppp_finalize(h)          # reductions only: the replica state stays as advanced
        torch.cuda.synchronize()
        tim = ppp.ppp_get_timings(h)
        blob = ppp.ppp_checkpoint(h)
    finally:
        ppp.ppp_destroy(h)
    assert int(np.frombuffer(blob, dtype=np.int64, count=1, offset=8)[0]) == steps
    n_pad = int(tim["variant_lanes"]) * int(tim["variant_beads_per_lane"])
    n_rep = len(prob["lambda"]) * prob["n_replicas"]
    state = np.frombuffer(blob, dtype=np.float32, count=n_rep * 6 * n_pad, offset=16).reshape(n_rep, 6, n_pad)
    n = prob["n_beads"]
    out = {}
    for gid in picks:
        out[gid] = state[gid, 0:3, :n].T.astype(np.float64)
    return out, (tim["variant_lanes"], tim["variant_beads_per_lane"])


def _check(prob, steps, picks, name):
    got, shape = _run_and_sample(prob, steps, picks)
    R = prob["n_replicas"]
    worst = 0.0
    for gid, x in got.items():
        w, r = divmod(gid, R)
        ref = oracle.trajectory(dict(prob, precision="fp64"), w, r, steps)[-1].reshape(-1, 3)
        err = float(np.max(np.abs(x - ref)))
        worst = max(worst, err)
        assert err < 1e-4, (name, gid, err)
    _say(f"  {name} (shape {shape[0]}x{shape[1]}): {len(picks)} sampled replicas after {steps} steps, "
         f"max |x_gpu - x_oracle| = {worst:.2e}")


def test_chain10_full_size_sampled_replicas():
    prob = ppp_inputs.config_chain10()
    _say("case full-size chain10: 21 windows x 1024 replicas, one launch of 20 steps")
    # items hold 48 consecutive replicas (5x2 shape, 12 per wavefront); window 1 starts at 1024
    _check(prob, 20, [0, 47, 48, 1023, 1024, 10 * 1024 + 517, 21 * 1024 - 1], "chain10")


def test_chain256_full_size_sampled_replicas():
    prob = ppp_inputs.config_chain256()
    _say("case full-size chain256: 41 windows x 4096 replicas, one launch of 5 steps")
    # items hold 4 consecutive replicas (64x4 shape, one per wavefront); window 1 starts at 4096
    _check(prob, 5, [0, 3, 4, 4095, 4096, 20 * 4096 + 1234, 41 * 4096 - 1], "chain256")


def test_chain32_full_size_sampled_replicas():
    prob = ppp_inputs.config_chain32()
    _say("case full-size chain32: 21 windows x 4096 replicas, one launch of 10 steps")
    # items hold 16 consecutive replicas (16x2 shape, 4 per wavefront); window 1 starts at 4096
    _check(prob, 10, [0, 15, 16, 4095, 4096, 13 * 4096 + 2222, 21 * 4096 - 1], "chain32")


def test_chain256_full_size_chunked_advance_is_bit_identical():
    """The bench times the 256-bead workload in chunks of one launch each; the
    state after 6 steps in one launch and after 2 + 4 steps in two launches
    (41 x 4096 replicas, fp32) is the same to the last bit: every replica's
    positions and velocities, its accumulators and the histograms."""
    prob = ppp_inputs.config_chain256()
    _say("case full-size chain256: 6 steps in one launch against 2 + 4 in two")
    blobs = []
    for chunks in ([6], [2, 4]):
        h = ppp.ppp_create(prob)
        try:
            ws = ppp.workspace(h)
            ppp.ppp_begin(h, ws)
            for c in chunks:
                ppp.ppp_advance(h, c)
            torch.cuda.synchronize()
            blobs.append(ppp.ppp_checkpoint(h))
            del ws
        finally:
            ppp.ppp_destroy(h)
    a, b = (np.frombuffer(x, dtype=np.uint8) for x in blobs)
    assert a.size == b.size and a.size > 10**9          # 167936 replicas x 6 x 256 fp32 = 1.03e9 B of state
    diff = int(np.count_nonzero(a != b))
    _say(f"  {a.size / 1e9:.3f} GB of state, accumulators and histograms; bytes that differ: {diff}")
    assert diff == 0


def test_batch_full_size_matches_single_runs():
    """The uneven batch at full size (64 chains, 2.7e10 replica-steps) in the one
    graph launch `bench.py --workload batch` times: the cheapest problem of each
    chain-length class (up to 8, 12, 16, 32, 64 and 128 beads, so each kernel
    shape group of the graph is sampled) reproduces its own single run bit for
    bit in every output, and no replica of the batch is frozen.  A replica run on
    another problem's parameters, noise stream or window, or an item that a
    persistent workgroup skipped or ran twice, changes these outputs."""
    probs = ppp_inputs.batched_instances()
    edges = (8, 10, 12, 16, 32, 64, 128)
    pick = {}
    for i, p in enumerate(probs):
        n = p["n_beads"]
        cls = next(e for e in edges if n <= e)
        cost = len(p["lambda"]) * p["n_replicas"] * p["n_steps"] * n * n
        if cls not in pick or cost < pick[cls][1]:
            pick[cls] = (i, cost)
    sample = sorted(i for i, _ in pick.values())
    _say(f"case full-size batch: 64 chains in one graph; sampled problems {sample} "
         f"(beads {[probs[i]['n_beads'] for i in sample]})")
    h = ppp.ppp_batch_create(probs)
    try:
        ws = ppp.workspace(h)
        ppp.ppp_run(h, ws)
        torch.cuda.synchronize()
        _say(f"  graph: {ppp.ppp_get_timings(h)['sim_ms']:.0f} ms")
        batch = {i: ppp.ppp_batch_get_result(h, probs[i], i) for i in range(len(probs))}
        del ws
    finally:
        ppp.ppp_destroy(h)
    frozen = sum(int(np.sum(r["n_blown_up"])) for r in batch.values())
    assert frozen == 0, frozen
    keys = ("dF_je", "dF_fluct", "dF_gauss", "dF_je_se", "xi_mean", "xi_std", "n_samples", "xi_hist",
            "dF_je_hist", "work_hist", "overlap_ovl", "kish_frac", "work_hist_rev", "dF_crooks", "sigma_lsq")
    for i in sample:
        single = ppp.run(probs[i])[0]
        for key in keys:
            a, b = np.asarray(batch[i][key]), np.asarray(single[key])
            same = np.array_equal(a, b, equal_nan=True) if np.issubdtype(a.dtype, np.floating) \
                else np.array_equal(a, b)
            assert same, (i, key)
    _say(f"  {len(sample)} problems equal to their single runs in {len(keys)} outputs each")
