"""Throughput benchmark of the parallel pulling protocol on one MI355X.

Default workload: the 256-bead chain (41 windows x 4096 replicas, all
Lennard-Jones pairs), the configuration the fp32 roofline target is set on.
A whole run is 200000 steps (about eight minutes), so one bench step is one
chunk of it: ppp_advance by --chunk steps of every replica of every window
(force evaluation, noise, BAOAB, sampling and fp64 accumulation), then
ppp_finalize (reductions, estimators, App. C work distributions) on what has
been sampled so far.  The initial state is built untimed before the warm-up
steps; inputs stay resident in device memory.  `value` is replica-steps
(one integrator step of one replica) per second of wall time over the timed
steps.  Smaller workloads (--workload chain10, ...) run whole passes of the
protocol per step.

Extra keys: the dF error at equal budget (uniform, learned and no-network
window placement against a dense reference run, 32-bead chain) and the
10-bead workload's whole-pass rate as a secondary line.

Prints one JSON line.  --gpus N with N > 1 exits: the protocol runs on one GPU here.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("replica-steps/sec and ΔF abs error (kT) at equal budget: plain vs batched+learned windows")
FP32_PEAK = 157.3e12     # MI355X fp32 vector, TFLOP/s (packed); unpacked FMA peak is half
FP64_PEAK = 78.6e12


# HBM traffic of one launch of the simulation kernel, from two rocprofv3 --pmc runs of
# this script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
# same counter reads for a 1 GiB device-to-device copy in the same run (--pmc-copy-mib
# 1024): the copy reads 1048576 KiB and writes as much, so a scale is 1048576 over the
# copy's reading.  chain256: the second of two launches of 1000 steps (--profile-launches
# 2), which reads the state the first one wrote, as every timed launch does.
# A record holds only while the kernel sources hash to the digest it was taken on.
TRAFFIC = {
    "chain256": {"sources_sha1": "132d8b7818ff4fe038531f59df1060b7b3448968", "kernel": "sim_chain<float,64,4>",
                 "fetch_kib": 517151.0, "fetch_scale": 1048576 / 524315.9375, "write_kib": 1028608.0,
                 "write_scale": 1048576 / 1048576.0},
    "chain10": {"sources_sha1": "132d8b7818ff4fe038531f59df1060b7b3448968", "kernel": "sim_chain<float,5,2>",
                "fetch_kib": 169.0, "fetch_scale": 1048576 / 524308.125, "write_kib": 10145.71875,
                "write_scale": 1048576 / 1048576.0},
}
KERNEL_SOURCES = ("ppp_sim_impl.hpp", "ppp_chain_force.hpp", "ppp_device.hpp", "ppp_internal.hpp", "ppp_sim.hip",
                  "ppp_shapes.hpp", "ppp_launch.hpp")


def kernel_sources_digest():
    import hashlib
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1105_4840_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """Bytes per launch from the counter record, or None when it does not apply."""
    rec = TRAFFIC.get(workload)
    if rec is None or rec["kernel"] != kernel or rec["sources_sha1"] != kernel_sources_digest():
        return None
    return 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])


def chain_flops_per_replica_step(n_beads):
    """Algorithmic fp32 flops of one replica-step of the chain: 24 per non-excluded
    Lennard-Jones pair (all |i-j| > 2 pairs are evaluated), 21 per bond, 45 per
    angle, 11 per mobile degree of freedom (BAOAB) and 15 for the restraint."""
    n = n_beads
    pairs = max(0, n * (n - 1) // 2 - (n - 1) - max(0, n - 2))
    return 24 * pairs + 21 * (n - 1) + 45 * max(0, n - 2) + 11 * 3 * (n - 1) + 15


WORKLOADS = {
    "chain10": ("config_chain10", "10-bead chain (bonds k_b=100, cosine angles k_theta=5, LJ eps=sigma=1 rc=2.5), "
                "end-to-end restraint k=20, 21 windows in [1.5, 8.5], 1024 replicas/window, 40000 BAOAB steps "
                "dt=0.005 kT=1, fp32 forces/integration, fp64 work/LSE/estimators"),
    "chain32": ("config_chain32", "32-bead chain, same force field, k=20, 21 uniform windows in [3, 28], "
                "4096 replicas/window, 23251 steps (2e9 replica-steps)"),
    "chain256": ("config_chain256", "256-bead chain (bonds k_b=100, cosine angles k_theta=5, LJ eps=sigma=1 "
                 "rc=2.5, all pairs |i-j|>2 evaluated), end-to-end restraint k=20 pulled from the helix over the "
                 "first 10000 steps, 41 windows in [10, 200], 4096 replicas/window, 200000 BAOAB steps dt=0.005 "
                 "kT=1, fp32 forces/integration, fp64 work/LSE/estimators"),
    "batch": ("batched_instances", "64 independent chains in one persistent, graph-captured launch: lengths "
              "U{8..128}, 11-41 windows, 64-1024 replicas/window, 5e3-1e5 steps (log-uniform), same force field, "
              "k=20, fp32 forces/fp64 work"),
    "1d": ("config_1d", "1-D double well U=5(x^2-1)^2, k=50, 21 windows in [-1.5, 1.5], 256 replicas/window, "
           "20000 overdamped LM steps dt=1e-3, fp64"),
}


# steps per bench step for workloads too long for one pass per step
DEFAULT_CHUNK = {"chain256": 1000}


def cpu_baseline(prob, target_seconds):
    """The fp64 oracle on a bounded sample of the same workload: every window and the
    full per-replica step count with fewer replicas; where even two replicas would run
    well past the target time (the long chains), fewer steps as well.  A shortened run
    keeps the equilibration share of the steps; where the centre is pulled, the pull
    and the equilibration take the first two thirds of the sample's steps (a pull
    scaled down with the steps would be faster than the chain can follow and freeze
    replicas, which the oracle then stops early).  Replica-steps count the steps each
    replica actually ran."""
    import numpy as np
    import oracle
    n_win = len(prob["lambda"])

    def sized(reps, steps):
        p = dict(prob)
        p["n_replicas"] = int(reps)
        if steps < prob["n_steps"]:
            p["n_steps"] = int(steps)
            p["n_equil"] = int(steps) * int(prob["n_equil"]) // int(prob["n_steps"])
            if int(prob.get("n_pull", 0)) > 0:
                p["n_pull"] = p["n_equil"] = 2 * int(steps) // 3
        return p

    def steps_run(p, kept):
        # a frozen replica stops at the sample that froze it
        full = kept == oracle.samples_per_replica(p)
        ran = np.where(full, p["n_steps"], np.minimum(p["n_steps"], p["n_equil"] + (kept + 1) * p["sample_every"]))
        return int(ran.sum()), int((~full).sum())

    def parallel(items, threads):   # items run at once on average (dynamic schedule, equal items)
        return items / math.ceil(items / max(1, threads))

    # calibrate on a short sample, then size the measured one
    cal_steps = min(int(prob["n_steps"]), 3000)
    pc = sized(2, cal_steps)
    t0 = time.time(); _, kc, used = oracle.run(pc); t_cal = max(time.time() - t0, 1e-3)
    per_item = steps_run(pc, kc)[0] / t_cal / parallel(2 * n_win, used)   # replica-steps/s per thread
    steps = int(prob["n_steps"])
    reps = int(target_seconds * per_item * used / (n_win * steps))
    if reps < 2:
        steps = int(max(min(steps, 3000), min(steps, target_seconds * per_item * used / (n_win * 2))))
        reps = max(2, int(target_seconds * per_item * used / (n_win * steps)))
    reps = min(reps, int(prob["n_replicas"]))
    p = sized(reps, steps)
    t0 = time.time(); xi, kept, threads = oracle.run(p); el = time.time() - t0
    rs, frozen = steps_run(p, kept)
    pull = f", pull and equilibration over the first {p['n_pull']}" if int(p.get("n_pull", 0)) > 0 else ""
    return {"value": rs / el, "unit": "replica-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_win} windows x {reps} replicas x {p['n_steps']} steps{pull} "
                      f"({rs:.3g} replica-steps run, {frozen} replicas frozen, {el:.1f} s, fp64 C, "
                      f"OpenMP over replicas)",
            "host": host_cpu()}


def host_cpu():
    """CPU model and logical CPUs visible to this process, as the oracle timing's context."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def dF_error_block(args, log=True):
    """dF abs error at equal budget on the 32-bead chain, windows in [3, 28] (the
    workload of the learned part): against a dense, long reference run (201 windows,
    --ref-steps steps), the plain protocol with 21 uniform windows at the full budget
    of 2e9 replica-steps; learned placement at half and at the full budget; and, at
    the half budget, the two baselines that isolate what the surrogate adds: uniform
    windows at the count the learned placement chose, relaxing as long as its
    production windows, all of the budget in production; and the same exploration
    rounds and placement rule with sigma(lambda) interpolated from the explored
    windows' sample sigma_i (no network)."""
    import numpy as np
    import paper_1105_4840_amd as ppp
    import ppp_inputs

    def say(msg):
        if log:
            print(msg, file=sys.stderr, flush=True)

    def err(res, lam, ref_lam, ref, used, extra=None):
        out = {"windows": int(len(lam)), "replica_steps": int(used)}
        for key in ("dF_je", "dF_fluct", "dF_gauss", "dF_com"):
            f = np.interp(lam, ref_lam, ref["dF_je"])
            out[key + "_err_end"] = float(abs(res[key][-1] - ref["dF_je"][-1]))
            out[key + "_rms"] = float(np.sqrt(np.mean((res[key] - f) ** 2)))
        out["dF_je_se_end"] = float(res["dF_je_se"][-1])
        out["dl_over_sigma_max"] = float(np.nanmax(res["dlambda_over_sigma"]))
        out.update(extra or {})
        return out

    t0 = time.time()
    ref_p = ppp_inputs.config_chain32(n_windows=201, n_steps=args.ref_steps)
    ref, _ = ppp.run(ref_p)
    ref_lam = np.array(ref_p["lambda"])
    say(f"# dF block: reference 201 windows x 4096 x {args.ref_steps} steps, {time.time() - t0:.1f} s, "
        f"dF_je(28) = {ref['dF_je'][-1]:.3f} +- {ref['dF_je_se'][-1]:.3f}")
    budget = 21 * 4096 * 23251
    uni_p = ppp_inputs.config_chain32()
    uni, _ = ppp.run(uni_p)
    rows = {"uniform_21": err(uni, np.array(uni_p["lambda"]), ref_lam, ref, budget)}
    base = ppp_inputs.config_chain32(n_steps=4000)
    ad = {"initial_windows": 11, "max_rounds": 5, "max_windows": 256, "target_dl_over_sigma": 1.0,
          "train_iters": 800, "lr": 3e-3, "init_seed": 1, "explore_replicas": 256, "explore_steps": 2000,
          "min_production_steps": args.min_steps}
    for frac in (0.5, 1.0):
        res, lam, used = ppp.ppp_adaptive_run(base, dict(ad, budget_replica_steps=int(frac * budget)))
        rows[f"learned_{frac:g}budget"] = err(res, lam, ref_lam, ref, used)
        say(f"# dF block: learned at {frac:g} budget, {len(lam)} windows, {time.time() - t0:.1f} s")
        if frac == 0.5:
            # uniform windows at the learned count, each relaxing as long as a learned
            # production window (--min-steps), the replicas sized to spend the budget
            W = len(lam)
            steps = args.min_steps
            reps = min(4096, int(0.5 * budget) // (W * steps))
            steps = int(0.5 * budget) // (W * reps)
            up = ppp_inputs.config_chain32(n_replicas=reps, n_steps=steps, lam=np.linspace(3.0, 28.0, W))
            u, _ = ppp.run(up)
            rows["uniform_at_learned_count_0.5budget"] = err(u, np.array(up["lambda"]), ref_lam, ref,
                                                              W * reps * steps, {"steps": steps, "replicas": reps})
            e, lam_e, used_e = ppp.ppp_adaptive_run(base, dict(ad, budget_replica_steps=int(0.5 * budget),
                                                               placement="explored"))
            rows["explored_sigma_0.5budget"] = err(e, lam_e, ref_lam, ref, used_e)
            say(f"# dF block: baselines at 0.5 budget ({W} uniform, {len(lam_e)} explored-sigma windows), "
                f"{time.time() - t0:.1f} s")
    return {"workload": "32-bead chain, same force field, k=20, lambda in [3, 28], 4096 replicas/window, "
                        "budget 2e9 replica-steps",
            "reference": {"windows": 201, "steps": args.ref_steps, "dF_je_end": float(ref["dF_je"][-1]),
                          "dF_je_se_end": float(ref["dF_je_se"][-1]),
                          "dF_fluct_end": float(ref["dF_fluct"][-1]), "dF_gauss_end": float(ref["dF_gauss"][-1])},
            "rows": rows, "seconds": time.time() - t0}


def placement_study(args):
    print(json.dumps({"study": "dF abs error (kT) at equal budget", **dF_error_block(args)}), flush=True)


def batch_bench(args, desc):
    """The uneven batch: every problem in one graph launch (persistent kernels per
    kernel shape on side streams, then reductions, estimators and App. C)."""
    import numpy as np
    import torch
    import paper_1105_4840_amd as ppp
    import ppp_inputs
    probs = ppp_inputs.batched_instances()
    table = None
    if args.tune:
        import tempfile
        table = os.path.join(tempfile.mkdtemp(), "tune.txt")
        tws = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        st = ppp.lib().ppp_autotune(table.encode(), ppp._ptr(tws), tws.numel(), ppp._stream())
        if st != ppp.PPP_OK:
            raise RuntimeError(f"ppp_autotune: {ppp.lib().ppp_status_string(st)}")
        del tws
        print("# autotune done", file=sys.stderr, flush=True)
    h = ppp.ppp_batch_create(probs, table)
    ws = ppp.workspace(h)
    rs_per_run = sum(len(p["lambda"]) * p["n_replicas"] * p["n_steps"] for p in probs)
    flops = sum(len(p["lambda"]) * p["n_replicas"] * p["n_steps"] * chain_flops_per_replica_step(p["n_beads"])
                for p in probs)
    for i in range(args.warmup):
        ppp.ppp_run(h, ws)
        torch.cuda.synchronize()
        print(f"# warmup run {i + 1} done", file=sys.stderr, flush=True)
    graph_ms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ppp.ppp_run(h, ws)
        torch.cuda.synchronize()
        graph_ms.append(ppp.ppp_get_timings(h)["sim_ms"])
        print(f"# run {i + 1} done: {graph_ms[-1]:.1f} ms", file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    frozen = 0; worst = 0.0
    for i, p in enumerate(probs):
        r = ppp.ppp_batch_get_result(h, p, i)
        frozen += int(r["n_blown_up"].sum())
        worst = max(worst, float(np.max(r["n_blown_up"] / p["n_replicas"])))
    tim = ppp.ppp_get_timings(h)
    ppp.ppp_destroy(h)
    avg_s = float(np.mean(graph_ms)) * 1e-3
    out = {
        "metric": METRIC, "value": rs_per_run * args.steps / el, "unit": "replica-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch", "description": desc, "problems": len(probs),
                   "replica_steps_per_step": rs_per_run, "tune_table": bool(args.tune), "parallelism": "1 GPU"},
        "graph_replica_steps_per_s": rs_per_run / avg_s,
        "accuracy": {"frozen_replicas": frozen, "worst_window_frozen_fraction": worst},
        # the graph holds one persistent kernel per kernel shape, run concurrently; the
        # achieved rate is the whole graph's (reductions included, < 1% of it)
        "roofline": {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP32_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": flops / avg_s / FP32_PEAK, "traffic": None,
                     "kernel": "sim_chain_persistent<float,G,B> (all shapes, one graph)",
                     "flops_per_run": flops, "avg_launch_ms": avg_s * 1e3},
        "timings_ms": {"graph": tim["sim_ms"], "total": tim["total_ms"]},
    }
    print(json.dumps(out), flush=True)


def sweep_study(args):
    """Relaxation time and stiffness sweep (the analogues of the paper's tau and k
    studies, Sec. IV C-D) on the 10-bead chain, every problem in one batched graph:
    tau = 500 .. 40000 steps at k = 20, and k = 2 .. 200 at tau = 20000 steps, 21
    windows in [1.5, 8.5], 4096 replicas per window."""
    import numpy as np
    import torch
    import paper_1105_4840_amd as ppp
    import ppp_inputs
    taus = [500, 1000, 2000, 5000, 10000, 20000, 40000]
    ks = [2.0, 5.0, 10.0, 20.0, 50.0, 100.0, 200.0]
    probs, labels = [], []
    for t in taus:
        p = ppp_inputs.config_chain10(n_replicas=4096, n_steps=t, seed=11)
        probs.append(p); labels.append({"tau_steps": t, "k": 20.0})
    for k in ks:
        p = ppp_inputs.config_chain10(n_replicas=4096, n_steps=20000, seed=12)
        p["k"] = k
        probs.append(p); labels.append({"tau_steps": 20000, "k": k})
    h = ppp.ppp_batch_create(probs)
    ws = ppp.workspace(h)
    t0 = time.perf_counter()
    ppp.ppp_run(h, ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rows = []
    for i, (p, lab) in enumerate(zip(probs, labels)):
        r = ppp.ppp_batch_get_result(h, p, i)
        rows.append(dict(lab, dF_je=float(r["dF_je"][-1]), dF_je_se=float(r["dF_je_se"][-1]),
                         dF_fluct=float(r["dF_fluct"][-1]), dF_gauss=float(r["dF_gauss"][-1]),
                         dF_com=float(r["dF_com"][-1]), unc=float(r["dF_unc"][-1]),
                         gamma2_mean=float(np.mean(r["gamma2"])),
                         dl_over_sigma_max=float(np.max(r["dlambda_over_sigma"])),
                         ovl_min=float(np.min(r["overlap_ovl"])), kish_min=float(np.min(r["kish_frac"])),
                         criterion_ok=int(np.sum(r["criterion_ok"])), frozen=int(r["n_blown_up"].sum())))
    ppp.ppp_destroy(h)
    rs = sum(len(p["lambda"]) * p["n_replicas"] * p["n_steps"] for p in probs)
    print(json.dumps({"study": "tau and k sweep, 10-bead chain, 21 windows in [1.5, 8.5], 4096 replicas/window, "
                               "one batched graph", "replica_steps": rs, "seconds": el, "rows": rows}), flush=True)


def turn_on_study(args):
    """Turn-on free energy (Sec. II, Eqs. 5-7, 10, 15) with the unrestrained ensemble
    run beside the windows: the 10-bead chain workload (fp32 forces), and the 1-D
    double well in two settings, the bench one (U = 5 (x^2 - 1)^2, k = 50, windows
    in [-1.5, 1.5]), where the restrained window never visits the far well, and a
    shallow one (U = (x^2 - 1)^2, k = 2), where it does."""
    import numpy as np
    import torch
    import paper_1105_4840_amd as ppp
    import ppp_inputs
    rows = []
    p = ppp_inputs.config_chain10(n_replicas=1024, n_steps=40000, seed=21)
    p["free_ensemble"] = True
    t0 = time.perf_counter()
    r, tim = ppp.run(p)
    torch.cuda.synchronize()
    rows.append({"case": "chain10 fp32", "seconds": time.perf_counter() - t0, "replica_steps": tim["replica_steps"],
                 "turn_on": r["turn_on"], "dF_je_end": float(r["dF_je"][-1]), "G_end": float(r["G"][-1]),
                 "G_se_end": float(r["G_se"][-1])})
    for name, a, k, lam in (("1d double well a=5 k=50", 5.0, 50.0, (-1.5, 1.5)),
                            ("1d double well a=1 k=2", 1.0, 2.0, (-1.2, 0.9))):
        q = ppp_inputs.config_1d(n_replicas=1024, n_steps=40000, n_windows=21, seed=22)
        q.update({"pot_a": a, "k": k, "free_ensemble": True, "lambda": list(np.linspace(lam[0], lam[1], 21))})
        r, tim = ppp.run(q)
        rows.append({"case": name, "replica_steps": tim["replica_steps"], "turn_on": r["turn_on"],
                     "dF_je_end": float(r["dF_je"][-1])})
    print(json.dumps({"study": "turn-on free energy", "rows": rows}), flush=True)


def peak_study(args):
    """Measured ceilings beside the published ones, as context for the roofline
    fractions (which always use the published peaks): the fp32 FMA issue rate of
    plain (non-packed) v_fma_f32, the form every kernel here is compiled to, and a
    device-to-device copy for HBM."""
    import torch
    import paper_1105_4840_amd as ppp
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    n_blocks, iters = 16384, 16384
    out = torch.empty(n_blocks * 256, dtype=torch.float32, device=dev)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    flops = 16.0 * iters * n_blocks * 256
    fma_ms = {}
    for vgpr in (False, True):
        ppp.ppp_probe_valu(n_blocks, 64, out=out, vgpr_operands=vgpr)       # warm-up
        torch.cuda.synchronize()
        ms = []
        for _ in range(5):
            t0.record(stream)
            ppp.ppp_probe_valu(n_blocks, iters, out=out, stream=stream, vgpr_operands=vgpr)
            t1.record(stream)
            t1.synchronize()
            ms.append(t0.elapsed_time(t1))
        fma_ms[vgpr] = min(ms)
    fma = flops / (fma_ms[False] * 1e-3) / 1e12
    fma_v = flops / (fma_ms[True] * 1e-3) / 1e12
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    cms = []
    for _ in range(10):
        t0.record(stream)
        dst.copy_(src)
        t1.record(stream)
        t1.synchronize()
        cms.append(t0.elapsed_time(t1))
    gbs = 2.0 * nbytes / (min(cms) * 1e-3) / 1e9
    print(json.dumps({
        "study": "measured ceilings (context; roofline fractions use the published peaks)",
        "fp32_fma": {"tflops": fma, "ms": fma_ms[False], "operands": "b, c in scalar registers",
                     "flops": flops, "threads": n_blocks * 256, "chains_per_thread": 8,
                     "published_packed_peak": FP32_PEAK / 1e12, "published_unpacked_rate": FP32_PEAK / 2e12,
                     "frac_of_unpacked": fma / (FP32_PEAK / 2e12), "frac_of_peak": fma / (FP32_PEAK / 1e12)},
        "fp32_fma_vgpr": {"tflops": fma_v, "ms": fma_ms[True], "operands": "b, c in vector registers",
                          "frac_of_peak": fma_v / (FP32_PEAK / 1e12),
                          "cycles_per_wave_instruction": 1024 * 2.4e9 * fma_ms[True] * 1e-3 / (flops / 128.0)},
        "hbm_copy": {"gb_per_s": gbs, "ms": min(cms), "bytes_moved": 2 * nbytes, "published_peak": 8000.0,
                     "frac": gbs / 8000.0},
    }))


def chunked_bench(args, prob, desc, stream):
    """One bench step = ppp_advance by args.chunk steps + ppp_finalize (see the module
    docstring); the initial state is built before the warm-up steps."""
    import numpy as np
    import torch
    import paper_1105_4840_amd as ppp
    n_win = len(prob["lambda"])
    need = (args.warmup + args.steps) * args.chunk
    if need > prob["n_steps"]:
        raise SystemExit(f"bench.py: (warmup + steps) x chunk = {need} exceeds the workload's "
                         f"{prob['n_steps']} steps; lower --chunk")
    h = ppp.ppp_create(prob)
    ws = ppp.workspace(h)
    ppp.ppp_begin(h, ws, stream)
    torch.cuda.synchronize()

    def one_step():
        ppp.ppp_advance(h, args.chunk, stream)
        ppp.ppp_finalize(h, stream)

    for i in range(args.warmup):
        one_step()
        torch.cuda.synchronize()
        print(f"# warmup step {i + 1}: {ppp.ppp_steps_done(h)} steps done", file=sys.stderr, flush=True)
    adv_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step()
        tim = ppp.ppp_get_timings(h)       # HIP events on the launch stream (synchronises it)
        adv_ms.append(tim["last_advance_ms"])
        print(f"# step {i + 1}: advance {adv_ms[-1]:.1f} ms, {ppp.ppp_steps_done(h)} steps done", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = ppp.ppp_get_result(h, prob)
    tim = ppp.ppp_get_timings(h)
    done = ppp.ppp_steps_done(h)
    ppp.ppp_destroy(h)
    rs_step = n_win * prob["n_replicas"] * args.chunk
    avg_s = float(np.mean(adv_ms)) * 1e-3
    flops = chain_flops_per_replica_step(prob["n_beads"]) * rs_step
    kname = f"sim_chain<float,{tim['variant_lanes']},{tim['variant_beads_per_lane']}>"
    dls = np.asarray(res["dlambda_over_sigma"])
    out = {
        "metric": METRIC, "value": rs_step * args.steps / el, "unit": "replica-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "protocol": "parallel", "description": desc, "windows": n_win,
                   "replicas_per_window": prob["n_replicas"], "relaxation_steps": prob["n_steps"],
                   "steps_per_bench_step": args.chunk, "replica_steps_per_step": rs_step,
                   "bench_step": "ppp_advance(chunk) + ppp_finalize (reductions, estimators, App. C)",
                   "parallelism": "1 GPU"},
        "kernel_replica_steps_per_s": rs_step / avg_s,
        "phase_ms": {"advance": float(np.mean(adv_ms)), "reduce_estimators": tim["reduce_ms"],
                     "appc": tim["appc_ms"]},
        # what the run has computed when the timed steps end: the first `done` of the
        # workload's steps, sampled from n_equil on; the builder's full runs are in DESIGN
        "accuracy": {
            "steps_done": int(done), "samples_per_replica": int(res["n_samples"][0] // prob["n_replicas"]),
            "dF_je_end": float(res["dF_je"][-1]), "dF_je_se_end": float(res["dF_je_se"][-1]),
            "dF_fluct_end": float(res["dF_fluct"][-1]), "dF_fluct_se_end": float(res["dF_fluct_se"][-1]),
            "dF_gauss_end": float(res["dF_gauss"][-1]), "dF_com_unc_end": float(res["dF_unc"][-1]),
            "dlambda_over_sigma_max": float(np.nanmax(dls)) if dls.size else None,
            "dlambda_over_sigma_median": float(np.nanmedian(dls)) if dls.size else None,
            "criterion_ok": int(np.sum(res["criterion_ok"])), "criterion_pairs": int(n_win - 1),
            "frozen_replicas": int(res["n_blown_up"].sum()),
            "note": "41 uniform windows at k=20 lie far more than 3 sigma apart (see dlambda_over_sigma): the "
                    "forward work distributions do not overlap and dF_je rests on unsampled tails (the "
                    "failure mode of Sec. IV B); dF_fluct (Eq. 14) is the usable estimate here"},
        "roofline": {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP32_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": flops / avg_s / FP32_PEAK,
                     "traffic": measured_traffic(args.workload, kname), "kernel": kname,
                     "flops_per_replica_step": chain_flops_per_replica_step(prob["n_beads"]),
                     "avg_launch_ms": avg_s * 1e3, "launches_per_step": 1},
    }
    return out


def whole_pass_bench(args, prob, stream, steps, warmup):
    """One bench step = one whole pass (ppp_run: initial state, every relaxation step,
    reductions, estimators, App. C); returns the line's core fields."""
    import numpy as np
    import torch
    import paper_1105_4840_amd as ppp
    h = ppp.ppp_create(prob)
    ws = ppp.workspace(h)
    rs_per_run = len(prob["lambda"]) * prob["n_replicas"] * prob["n_steps"]
    steps_total = prob["n_steps"] * (len(prob["lambda"]) if prob.get("sequential") else 1)

    def one_run():
        if args.chunk and args.chunk > 0:
            ppp.ppp_begin(h, ws, stream)
            done = 0
            while done < steps_total:
                ppp.ppp_advance(h, args.chunk, stream)
                torch.cuda.synchronize()
                done = ppp.ppp_steps_done(h)
                print(f"# progress {done}/{steps_total} steps", file=sys.stderr, flush=True)
            ppp.ppp_finalize(h, stream)
        else:
            ppp.ppp_run(h, ws, stream)

    for _ in range(warmup):
        one_run()
    torch.cuda.synchronize()
    sim_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        one_run()
        sim_ms.append(ppp.ppp_get_timings(h)["sim_ms"])   # HIP events on the launch stream
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = ppp.ppp_get_result(h, prob)
    tim = ppp.ppp_get_timings(h)
    ppp.ppp_destroy(h)
    launches = max(1, int(tim["sim_launches"]))
    avg_sim_s = float(np.mean(sim_ms)) * 1e-3 / launches
    rs_per_launch = rs_per_run / launches
    if prob["model"] == "chain":
        flops = chain_flops_per_replica_step(prob["n_beads"]) * rs_per_launch
        kname = f"sim_chain<float,{tim['variant_lanes']},{tim['variant_beads_per_lane']}>"
        roof = {"bound": "alu", "achieved": flops / avg_sim_s / 1e12, "peak": FP32_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": flops / avg_sim_s / FP32_PEAK,
                "traffic": measured_traffic(prob.get("name"), kname),
                "kernel": kname, "flops_per_replica_step": chain_flops_per_replica_step(prob["n_beads"]),
                "avg_launch_ms": avg_sim_s * 1e3, "launches_per_step": launches}
    else:
        flops = 12 * rs_per_launch
        roof = {"bound": "alu", "achieved": flops / avg_sim_s / 1e12, "peak": FP64_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": flops / avg_sim_s / FP64_PEAK, "traffic": None,
                "kernel": "sim_1d<double>", "flops_per_replica_step": 12, "avg_launch_ms": avg_sim_s * 1e3}
    return {
        "value": rs_per_run * steps / el, "ms_per_step": el / steps * 1e3, "replica_steps_per_step": rs_per_run,
        "kernel_replica_steps_per_s": rs_per_launch / avg_sim_s,
        "phase_ms": {"sim": tim["sim_ms"], "reduce_estimators": tim["reduce_ms"], "appc": tim["appc_ms"]},
        "accuracy": {"dF_je_end": float(res["dF_je"][-1]), "dF_je_se_end": float(res["dF_je_se"][-1]),
                     "dF_fluct_end": float(res["dF_fluct"][-1]), "dF_com_unc_end": float(res["dF_unc"][-1]),
                     "frozen_replicas": int(res["n_blown_up"].sum())},
        "roofline": roof,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="chain256", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="leave out the dF-at-equal-budget block and the secondary 10-bead line")
    ap.add_argument("--chunk", type=int, default=None,
                    help="steps per bench step (chunked workloads) or per advance (progress lines)")
    ap.add_argument("--placement-study", action="store_true",
                    help="dF error at equal budget, uniform vs learned windows (32-bead chain), alone")
    ap.add_argument("--ref-steps", type=int, default=40000)
    ap.add_argument("--sweep", action="store_true", help="tau and k sweep of the 10-bead chain in one batched graph")
    ap.add_argument("--turn-on", action="store_true", help="turn-on free energy study (unrestrained ensemble)")
    ap.add_argument("--peak", action="store_true", help="measured fp32 FMA and HBM copy rates beside the published peaks")
    ap.add_argument("--min-steps", type=int, default=20000, help="relaxation steps per learned production window")
    ap.add_argument("--sequential", action="store_true",
                    help="run the workload with the sequential pulling protocol (each replica runs the "
                         "windows one after another; same replica-steps)")
    ap.add_argument("--profile-launches", type=int, default=0,
                    help="with --chunk: stop after this many advances and print no bench line "
                         "(for counter collection on one launch of a long workload)")
    ap.add_argument("--tune", action="store_true",
                    help="batch workload: run the autotuner first and use its table")
    ap.add_argument("--pmc-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the protocol runs on one GPU here; --gpus must be 1 (windows and replica "
              "blocks are independent, but no multi-GPU launch is implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1105_4840_amd as ppp
    import ppp_inputs

    torch.cuda.set_device(0)
    for flag, fn in ((args.placement_study, placement_study), (args.sweep, sweep_study),
                     (args.turn_on, turn_on_study), (args.peak, peak_study)):
        if flag:
            fn(args)
            return
    fn, desc = WORKLOADS[args.workload]
    stream = torch.cuda.current_stream()
    if args.workload == "batch":
        batch_bench(args, desc)
        return
    prob = getattr(ppp_inputs, fn)()
    if args.sequential:
        prob["sequential"] = True
    if args.pmc_copy_mib > 0:
        src = torch.ones(args.pmc_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.profile_launches > 0:
        chunk = args.chunk or DEFAULT_CHUNK.get(args.workload, 0)
        if chunk <= 0:
            raise SystemExit("--profile-launches needs --chunk")
        h = ppp.ppp_create(prob)
        ws = ppp.workspace(h)
        ppp.ppp_begin(h, ws, stream)
        for i in range(args.profile_launches):
            t0 = time.perf_counter()
            ppp.ppp_advance(h, chunk, stream)
            torch.cuda.synchronize()
            print(f"# profiled advance {i + 1}: {(time.perf_counter() - t0) * 1e3:.1f} ms wall", file=sys.stderr,
                  flush=True)
        ppp.ppp_destroy(h)
        return

    chunked = not args.sequential and (args.chunk or DEFAULT_CHUNK.get(args.workload, 0)) > 0 and \
        args.workload in DEFAULT_CHUNK
    if chunked:
        args.chunk = args.chunk or DEFAULT_CHUNK[args.workload]
        out = chunked_bench(args, prob, desc, stream)
    else:
        core = whole_pass_bench(args, prob, stream, args.steps, args.warmup)
        out = {
            "metric": METRIC, "value": core["value"], "unit": "replica-steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": core["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if prob.get("precision") == "fp64" else "f32",
            "data": "synthetic",
            "config": {"workload": args.workload + ("-sequential" if args.sequential else ""),
                       "protocol": "sequential" if args.sequential else "parallel",
                       "description": desc, "windows": len(prob["lambda"]),
                       "replicas_per_window": prob["n_replicas"], "relaxation_steps": prob["n_steps"],
                       "replica_steps_per_step": core["replica_steps_per_step"], "parallelism": "1 GPU"},
            "kernel_replica_steps_per_s": core["kernel_replica_steps_per_s"],
            "phase_ms": core["phase_ms"], "accuracy": core["accuracy"], "roofline": core["roofline"],
        }
    if not args.no_extras and args.workload == "chain256":
        # the 10-bead workload, whole passes (21 windows x 1024 replicas x 40000 steps)
        sec_args = argparse.Namespace(**dict(vars(args), chunk=0, workload="chain10"))
        p10 = ppp_inputs.config_chain10()
        core = whole_pass_bench(sec_args, p10, stream, 5, 1)
        out["secondary"] = {"chain10": {"description": WORKLOADS["chain10"][1], "steps": 5, "warmup": 1,
                                        **{k: core[k] for k in ("value", "ms_per_step", "kernel_replica_steps_per_s",
                                                                "accuracy", "roofline")}}}
        print(f"# secondary chain10 done: {core['value']:.4g} replica-steps/s", file=sys.stderr, flush=True)
        out["dF_error_at_equal_budget"] = dF_error_block(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
        out["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
