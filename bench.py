"""Throughput benchmark of the parallel pulling protocol on one MI355X.

One step = one whole pass of the protocol on one batch of synthetic input:
initial state, all relaxation steps of every replica of every window,
reductions, estimators (Eqs. 12-14, jackknife, overlap) and App. C work
distributions, with inputs resident in device memory.  `value` is the number
of replica-steps (one integrator step of one replica, with its force
evaluation, noise, sampling and accumulation) per second of wall time.

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
# 1024: FETCH_SIZE reads 529747.5 KiB -> x1.9794, WRITE_SIZE 1059107.1 KiB -> x0.9901).
# A record holds only while the kernel sources hash to the digest it was taken on.
TRAFFIC = {
    "chain10": {"sources_sha1": "04fdcc61e43361cc039f1648b793919ae0c4150d", "kernel": "sim_chain<float,5,2>",
                "fetch_kib": 175.0, "fetch_scale": 1.9794, "write_kib": 10146.03125, "write_scale": 0.9901},
}
KERNEL_SOURCES = ("ppp_sim_impl.hpp", "ppp_device.hpp", "ppp_internal.hpp", "ppp_sim.hip", "ppp_shapes.hpp",
                  "ppp_launch.hpp")


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
    "chain256": ("config_chain256", "256-bead chain, same force field, all LJ pairs, k=20, 41 windows in [10, 200], "
                 "4096 replicas/window, 200000 steps"),
    "batch": ("batched_instances", "64 independent chains in one persistent, graph-captured launch: lengths "
              "U{8..128}, 11-41 windows, 64-1024 replicas/window, 5e3-1e5 steps (log-uniform), same force field, "
              "k=20, fp32 forces/fp64 work"),
    "1d": ("config_1d", "1-D double well U=5(x^2-1)^2, k=50, 21 windows in [-1.5, 1.5], 256 replicas/window, "
           "20000 overdamped LM steps dt=1e-3, fp64"),
}


def cpu_baseline(prob, target_seconds):
    """The fp64 oracle on a bounded sample of the same workload: every window and the
    full per-replica step count with fewer replicas; where even two replicas would run
    well past the target time (the long chains), two replicas and fewer steps, with
    the equilibration and pulling phases scaled alike."""
    import oracle
    n_win = len(prob["lambda"])

    def sized(reps, steps):
        p = dict(prob)
        p["n_replicas"] = int(reps)
        if steps < prob["n_steps"]:
            p["n_steps"] = int(steps)
            p["n_equil"] = int(steps) * int(prob["n_equil"]) // int(prob["n_steps"])
            if int(prob.get("n_pull", 0)) > 0:
                p["n_pull"] = max(1, int(steps) * int(prob["n_pull"]) // int(prob["n_steps"]))
        return p

    def parallel(items, threads):   # items run at once on average (dynamic schedule, equal items)
        return items / math.ceil(items / max(1, threads))

    # calibrate on a short sample, then size the measured one
    cal_steps = min(int(prob["n_steps"]), 4000)
    t0 = time.time(); _, _, used = oracle.run(sized(2, cal_steps)); t_cal = max(time.time() - t0, 1e-3)
    per_item = 2 * n_win * cal_steps / t_cal / parallel(2 * n_win, used)   # replica-steps/s per thread
    steps = int(prob["n_steps"])
    reps = int(target_seconds * per_item * used / (n_win * steps))
    if reps < 2:
        reps = 2
        fit = target_seconds * per_item * parallel(2 * n_win, used) / (2 * n_win)
        steps = int(max(min(steps, 1000), min(steps, fit)))
    reps = min(reps, int(prob["n_replicas"]))
    p = sized(reps, steps)
    t0 = time.time(); xi, kept, threads = oracle.run(p); el = time.time() - t0
    rs = reps * n_win * p["n_steps"]
    return {"value": rs / el, "unit": "replica-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_win} windows x {reps} replicas x {p['n_steps']} steps "
                      f"({rs:.3g} replica-steps, {el:.1f} s, fp64 C, OpenMP over replicas)",
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


def placement_study(args):
    """dF error at equal budget, 32-bead chain, windows in [3, 28]: 21 uniform windows at
    2e9 replica-steps against learned placement at half (and at the full) budget; the
    reference is a dense, long run (201 windows, 40000 steps)."""
    import numpy as np
    import paper_1105_4840_amd as ppp
    import ppp_inputs

    def err(res, lam, ref_lam, ref):
        out = {}
        for key in ("dF_je", "dF_fluct", "dF_gauss", "dF_com"):
            f = np.interp(lam, ref_lam, ref["dF_je"])
            out[key + "_end"] = float(abs(res[key][-1] - ref["dF_je"][-1]))
            out[key + "_rms"] = float(np.sqrt(np.mean((res[key] - f) ** 2)))
        out["dF_je_se_end"] = float(res["dF_je_se"][-1])
        return out

    t0 = time.time()
    ref_p = ppp_inputs.config_chain32(n_windows=201, n_steps=args.ref_steps)
    ref, _ = ppp.run(ref_p)
    ref_lam = np.array(ref_p["lambda"])
    print(f"# reference: 201 windows x 4096 x {args.ref_steps} steps, {time.time() - t0:.1f} s, "
          f"dF_je(28) = {ref['dF_je'][-1]:.3f} +- {ref['dF_je_se'][-1]:.3f}", file=sys.stderr, flush=True)
    uni_p = ppp_inputs.config_chain32()
    uni, _ = ppp.run(uni_p)
    budget = 21 * 4096 * 23251
    rows = {"uniform_21": dict(err(uni, np.array(uni_p["lambda"]), ref_lam, ref), replica_steps=budget, windows=21)}
    for frac in (0.5, 1.0):
        base = ppp_inputs.config_chain32(n_steps=4000)
        ad = {"budget_replica_steps": int(frac * budget), "initial_windows": 11, "max_rounds": 5, "max_windows": 256,
              "target_dl_over_sigma": 1.0, "train_iters": 800, "lr": 3e-3, "init_seed": 1,
              "explore_replicas": 256, "explore_steps": 2000, "min_production_steps": args.min_steps}
        res, lam, used = ppp.ppp_adaptive_run(base, ad)
        rows[f"learned_{frac:g}budget"] = dict(err(res, lam, ref_lam, ref), replica_steps=used, windows=len(lam),
                                               dl_over_sigma_max=float(np.nanmax(res["dlambda_over_sigma"])))
        print(f"# learned at {frac:g} budget: {len(lam)} windows, {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    rows["uniform_21"]["dl_over_sigma_max"] = float(np.nanmax(uni["dlambda_over_sigma"]))
    print(json.dumps({"study": "dF abs error (kT) at equal budget, 32-bead chain, lambda in [3, 28]",
                      "reference": {"windows": 201, "steps": args.ref_steps, "dF_je_end": float(ref["dF_je"][-1]),
                                    "dF_je_se_end": float(ref["dF_je_se"][-1]),
                                    "dF_fluct_end": float(ref["dF_fluct"][-1]), "dF_gauss_end": float(ref["dF_gauss"][-1])},
                      "rows": rows}), flush=True)


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
    ppp.ppp_probe_valu(n_blocks, 64, out=out)                  # warm-up
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(5):
        t0.record(stream)
        ppp.ppp_probe_valu(n_blocks, iters, out=out, stream=stream)
        t1.record(stream)
        t1.synchronize()
        ms.append(t0.elapsed_time(t1))
    flops = 16.0 * iters * n_blocks * 256
    fma = flops / (min(ms) * 1e-3) / 1e12
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
        "fp32_fma": {"tflops": fma, "ms": min(ms), "flops": flops, "threads": n_blocks * 256, "chains_per_thread": 8,
                     "published_packed_peak": FP32_PEAK / 1e12, "published_unpacked_rate": FP32_PEAK / 2e12,
                     "frac_of_unpacked": fma / (FP32_PEAK / 2e12)},
        "hbm_copy": {"gb_per_s": gbs, "ms": min(cms), "bytes_moved": 2 * nbytes, "published_peak": 8000.0,
                     "frac": gbs / 8000.0},
    }))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chain10", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chunk", type=int, default=0, help="advance in chunks of this many steps (progress lines)")
    ap.add_argument("--placement-study", action="store_true",
                    help="dF error at equal budget, uniform vs learned windows (32-bead chain)")
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

    import numpy as np
    import torch
    import paper_1105_4840_amd as ppp
    import ppp_inputs

    if args.placement_study:
        torch.cuda.set_device(0)
        placement_study(args)
        return
    if args.sweep:
        torch.cuda.set_device(0)
        sweep_study(args)
        return
    if args.turn_on:
        torch.cuda.set_device(0)
        turn_on_study(args)
        return
    if args.peak:
        torch.cuda.set_device(0)
        peak_study(args)
        return
    fn, desc = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.workload == "batch":
        batch_bench(args, desc)
        return
    prob = getattr(ppp_inputs, fn)()
    if args.sequential:
        prob["sequential"] = True
    h = ppp.ppp_create(prob)
    ws = ppp.workspace(h)
    rs_per_run = len(prob["lambda"]) * prob["n_replicas"] * prob["n_steps"]

    # steps each replica takes (all windows in turn for the sequential protocol)
    steps_total = prob["n_steps"] * (len(prob["lambda"]) if args.sequential else 1)

    def one_run():
        if args.chunk > 0:
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

    if args.pmc_copy_mib > 0:
        src = torch.ones(args.pmc_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.profile_launches > 0:
        if args.chunk <= 0:
            raise SystemExit("--profile-launches needs --chunk")
        ppp.ppp_begin(h, ws, stream)
        for i in range(args.profile_launches):
            t0 = time.perf_counter()
            ppp.ppp_advance(h, args.chunk, stream)
            torch.cuda.synchronize()
            print(f"# profiled advance {i + 1}: {(time.perf_counter() - t0) * 1e3:.1f} ms wall", file=sys.stderr,
                  flush=True)
        ppp.ppp_destroy(h)
        return
    for _ in range(args.warmup):
        one_run()
    torch.cuda.synchronize()
    sim_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_run()
        t = ppp.ppp_get_timings(h)          # HIP events on the launch stream
        sim_ms.append(t["sim_ms"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = ppp.ppp_get_result(h, prob)
    tim = ppp.ppp_get_timings(h)
    ppp.ppp_destroy(h)

    value = rs_per_run * args.steps / el
    # per launch of the simulation kernel (a chunked run launches it once per advance)
    launches = max(1, int(tim["sim_launches"]))
    avg_sim_s = float(np.mean(sim_ms)) * 1e-3 / launches
    rs_per_launch = rs_per_run / launches
    if prob["model"] == "chain":
        flops = chain_flops_per_replica_step(prob["n_beads"]) * rs_per_launch
        kname = f"sim_chain<float,{tim['variant_lanes']},{tim['variant_beads_per_lane']}>"
        roof = {"bound": "alu", "achieved": flops / avg_sim_s / 1e12, "peak": FP32_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": flops / avg_sim_s / FP32_PEAK,
                "traffic": measured_traffic(args.workload, kname), "kernel": kname,
                "flops_per_replica_step": chain_flops_per_replica_step(prob["n_beads"]),
                "avg_launch_ms": avg_sim_s * 1e3, "launches_per_step": launches}
    else:
        flops = 12 * rs_per_launch
        roof = {"bound": "alu", "achieved": flops / avg_sim_s / 1e12, "peak": FP64_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": flops / avg_sim_s / FP64_PEAK, "traffic": None,
                "kernel": "sim_1d<double>", "flops_per_replica_step": 12, "avg_launch_ms": avg_sim_s * 1e3}
    out = {
        "metric": METRIC, "value": value, "unit": "replica-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prob.get("precision") == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload + ("-sequential" if args.sequential else ""),
                   "protocol": "sequential" if args.sequential else "parallel",
                   "description": desc, "windows": len(prob["lambda"]),
                   "replicas_per_window": prob["n_replicas"], "relaxation_steps": prob["n_steps"],
                   "replica_steps_per_step": rs_per_run, "parallelism": "1 GPU"},
        "kernel_replica_steps_per_s": rs_per_launch / avg_sim_s,
        "phase_ms": {"sim": tim["sim_ms"], "reduce_estimators": tim["reduce_ms"], "appc": tim["appc_ms"]},
        "accuracy": {"dF_je_end": float(res["dF_je"][-1]), "dF_je_se_end": float(res["dF_je_se"][-1]),
                     "dF_fluct_end": float(res["dF_fluct"][-1]), "dF_com_unc_end": float(res["dF_unc"][-1]),
                     "frozen_replicas": int(res["n_blown_up"].sum())},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
