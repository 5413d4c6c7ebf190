"""bench.py's host-side contract (no GPU): the one-GPU guard, the algorithmic
flop rule, the traffic record's digest check and the oracle baseline's fields."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import ppp_inputs  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("n", [2, 3, 4, 10, 32, 256])
def test_flop_rule_counts_every_pair_beyond_two_bonds(n):
    """24 per pair with |i-j| > 2 (counted here by enumeration), 21 per bond,
    45 per angle, 11 per mobile degree of freedom, 15 for the restraint."""
    pairs = sum(1 for i in range(n) for j in range(i + 1, n) if j - i > 2)
    want = 24 * pairs + 21 * (n - 1) + 45 * max(0, n - 2) + 11 * 3 * (n - 1) + 15
    assert bench.chain_flops_per_replica_step(n) == want
    if n == 10:
        assert want == 1533 and pairs == 28
    if n == 256:
        assert pairs == 32131 and want == 796359


def test_traffic_record_holds_only_for_its_kernel_and_sources(monkeypatch):
    rec = bench.TRAFFIC["chain10"]
    assert bench.measured_traffic("chain32", rec["kernel"]) is None
    assert bench.measured_traffic("chain10", "sim_chain<float,4,4>") is None
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: rec["sources_sha1"])
    got = bench.measured_traffic("chain10", rec["kernel"])
    assert got == pytest.approx(1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]))
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: "0" * 40)
    assert bench.measured_traffic("chain10", rec["kernel"]) is None


def test_oracle_baseline_reports_its_sample_and_host():
    prob = ppp_inputs.config_chain_small(4, n_replicas=8, n_steps=200, n_windows=3, precision="fp64")
    out = bench.cpu_baseline(prob, 0.2)
    assert out["kind"] == "oracle" and out["unit"] == "replica-steps/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "windows" in out["sample"] and "replicas" in out["sample"]
    assert out["host"]["logical_cpus"] >= 1


def test_chunked_bench_refuses_more_steps_than_the_workload_has():
    """A bench step of the 256-bead workload advances it by --chunk steps; asking
    for more steps than the run has is refused before any device work."""
    import argparse
    args = argparse.Namespace(warmup=5, steps=20, chunk=20000, workload="chain256")
    with pytest.raises(SystemExit) as e:
        bench.chunked_bench(args, ppp_inputs.config_chain256(), "", None)
    assert "exceeds" in str(e.value)


def test_oracle_baseline_keeps_a_pull_gentle_when_it_shortens_the_run():
    """Cut to fewer steps, a pulled run keeps the pull and the equilibration over the
    first two thirds of them and counts the steps its replicas actually ran."""
    prob = ppp_inputs.config_chain_small(4, n_replicas=4, n_steps=200000, n_windows=3, precision="fp64")
    prob["n_pull"] = 10000
    prob["n_equil"] = 20000
    out = bench.cpu_baseline(prob, 0.05)
    assert "pull and equilibration over the first" in out["sample"] and "0 replicas frozen" in out["sample"]
