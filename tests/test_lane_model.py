"""The chain kernels' lane layout on the CPU (no GPU): the device routines that
spread one replica over G lanes (forces, BAOAB step, lane moves, noise)
compiled for the host by tests/lane_model/lane_model.cpp, a wavefront as 64
threads exchanging through barriers, under AddressSanitizer and
UndefinedBehaviorSanitizer.  Every compiled kernel shape, and the
eight-beads-per-lane shapes the GPU build drops because they spill registers
there (16x8 among them), against the oracle: fp64 forces and energies within
1e-12, fp32 forces within 1e-5 at fp32-rounded coordinates, fp64 trajectories
within 1e-10; and no ds_permute destination written by two lanes."""
import concurrent.futures
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import ppp_inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "lane_model")
CSRC = os.path.join(ROOT, "paper_1105_4840_amd", "csrc")


def _gpu_shapes():
    import importlib.util
    spec = importlib.util.spec_from_file_location("ppp_pkg_build", os.path.join(ROOT, "paper_1105_4840_amd", "build.py"))
    build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(build)
    return build.shapes()


SPILLING = [(4, 8), (16, 8), (64, 8)]   # dropped from the GPU build (register spills)
SHAPES = _gpu_shapes() + SPILLING


@pytest.fixture(scope="module")
def models(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("lane_model")

    def build(shape):
        G, B = shape
        exe = str(out / f"lane_model_{G}x{B}")
        cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", "-Wno-unknown-pragmas", f"-DLM_G={G}", f"-DLM_B={B}", "-I", HERE,
               "-I", CSRC, "-I", os.path.join(ROOT, "include"), "-o", exe,
               os.path.join(HERE, "lane_model.cpp"), "-lpthread"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return shape, exe

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return dict(ex.map(build, SHAPES))


def _run(exe, mode, G, B, prec, prob, confs, n_steps=0, gid=0, centre=0.0):
    N = prob["n_beads"]
    head = f"{mode} {G} {B} {prec} {N} {len(confs)} {n_steps} {gid}\n"
    par = " ".join(repr(float(prob[k])) if k != "rc_mode" else str(int(prob[k]))
                   for k in ("k_bond", "r0", "k_angle", "lj_eps", "lj_sigma", "lj_rc", "rc_mode", "mass", "gamma",
                             "kT", "dt", "k"))
    body = "\n".join(" ".join(repr(float(v)) for v in c.ravel()) for c in confs)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], input=f"{head}{par} {centre!r} {int(prob['seed'])}\n{body}\n", capture_output=True,
                       text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    assert "permute conflicts 0" in r.stderr
    return np.array([float(x) for x in r.stdout.split()])


def _n_beads(G, B):
    return min(256, max(2, G * B - B // 2))   # padding beads in the last lane


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_lane_model_forces_match_oracle(models, shape):
    G, B = shape
    n = _n_beads(G, B)
    prob = ppp_inputs.config_chain_small(n, precision="fp64")
    confs = ppp_inputs.random_chain_coords(n, 2, seed=7 * G + B)
    lam = 0.4 * n
    out = _run(models[shape], 0, G, B, 64, prob, confs, centre=lam).reshape(len(confs), 3 * n + 5)
    for c in range(len(confs)):
        e, parts, fr = oracle.chain_forces(prob, confs[c], lam)
        f = out[c, :3 * n].reshape(n, 3)
        want = _without_restraint_on_bead0(prob, confs[c], lam, fr)
        assert np.linalg.norm(f - want) <= 1e-12 * np.linalg.norm(want)
        assert abs(out[c, 3 * n] - e) <= 1e-12 * abs(e)
    p32 = dict(prob, precision="fp32")
    c32 = confs.astype(np.float32).astype(np.float64)
    out = _run(models[shape], 0, G, B, 32, p32, c32, centre=lam).reshape(len(confs), 3 * n + 5)
    for c in range(len(confs)):
        _, _, fr = oracle.chain_forces(p32, c32[c], lam)
        f = out[c, :3 * n].reshape(n, 3)
        want = _without_restraint_on_bead0(p32, c32[c], lam, fr)
        assert np.linalg.norm(f - want) <= 1e-5 * np.linalg.norm(want)


def _without_restraint_on_bead0(prob, x, lam, fr):
    """The oracle's forces with the restraint's reaction on bead 0 taken off:
    bead 0 is held fixed, and the kernels leave that term out (its bonded and
    Lennard-Jones forces stay)."""
    want = np.array(fr, dtype=np.float64).reshape(-1, 3).copy()
    end = x[-1] - x[0]
    if prob.get("rc_mode", 0) == 1:
        xi, dxi = end[2], np.array([0.0, 0.0, 1.0])
    else:
        xi = np.linalg.norm(end)
        dxi = end / xi
    want[0] -= prob["k"] * (xi - lam) * dxi
    return want


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_lane_model_trajectory_matches_oracle(models, shape):
    """fp64 BAOAB steps through the kernel's own step routine, from the default
    helix with the kernel's step-0 velocities, against the oracle's trajectory of
    the same replica (fewer steps for the long chains: every exchange is a
    barrier of 64 threads here)."""
    G, B = shape
    n = _n_beads(G, B)
    steps = 100 if n <= 64 else 40
    prob = ppp_inputs.config_chain_small(n, n_replicas=4, n_steps=max(steps, 100), n_windows=3, precision="fp64")
    w, r = 2, 3
    gid = w * prob["n_replicas"] + r
    start = np.array(oracle.default_helix(n, prob["r0"])).reshape(1, n, 3)
    tr = _run(models[shape], 1, G, B, 64, prob, start, n_steps=steps, gid=gid,
              centre=prob["lambda"][w]).reshape(steps + 1, 3 * n)
    ref = oracle.trajectory(prob, w, r, steps)
    assert np.max(np.abs(tr - ref)) < 1e-10, np.max(np.abs(tr - ref))
