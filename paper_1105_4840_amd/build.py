"""Builds libppp.so (HIP kernels for gfx950 + the C-ABI runtime) in-tree with hipcc."""
import concurrent.futures
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libppp.so")
SOURCES = ["ppp_sim.hip", "ppp_reduce.hip", "ppp_mlp.hip", "ppp_probe.hip", "ppp_static.hip", "ppp_runtime.cpp",
           "ppp_adaptive.cpp"]
ARCH = os.environ.get("PPP_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed fp32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def shapes():
    """(G, B) chain-kernel shapes listed in csrc/ppp_shapes.hpp."""
    text = open(os.path.join(CSRC, "ppp_shapes.hpp")).read()
    body = text[text.index("PPP_FOR_EACH_SHAPE(X)"):]
    return [(int(g), int(b)) for g, b in re.findall(r"X\((\d+),\s*(\d+)\)", body)]


def _shape_sources():
    """One generated translation unit per (precision, shape) so they compile in parallel."""
    gen = os.path.join(OBJ, "gen")
    os.makedirs(gen, exist_ok=True)
    out = []
    for g, b in shapes():
        for t in ("float", "double"):
            name = f"shape_{t}_{g}x{b}.hip"
            text = ('#include "ppp_sim_impl.hpp"\n'
                    f"namespace ppp {{\nPPP_INSTANTIATE_SHAPE({t}, {g}, {b})\n}}\n")
            path = os.path.join(gen, name)
            if not os.path.exists(path) or open(path).read() != text:
                open(path, "w").write(text)
            out.append(path)
    return out


def _compile(src):
    path = src if os.path.isabs(src) else os.path.join(CSRC, src)
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    lang = ["-x", "hip"]
    cmd = ["hipcc", *lang, *COMMON, "-Rpass-analysis=kernel-resource-usage", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def _scratch_users(stderr):
    """Kernels of one translation unit that need scratch (spilled registers)."""
    bad, name = [], None
    for line in stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name and int(m.group(1)) > 0 and "sim_" in name:
            bad.append((name, int(m.group(1))))
    return bad


def build(verbose: bool = False) -> str:
    """Compiles every source (always) and links libppp.so; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = _shape_sources() + [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = int(os.environ.get("PPP_BUILD_JOBS", "8"))
    with concurrent.futures.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        results = list(ex.map(_compile, srcs))
    spills = [b for _, err in results for b in _scratch_users(err)]
    if spills:
        raise RuntimeError("simulation kernels spill to scratch (drop the shape from ppp_shapes.hpp): "
                           + ", ".join(f"{n} {b} B/lane" for n, b in spills))
    if verbose:
        for _, err in results:
            lines = [l for l in err.splitlines() if "remark" not in l and "Rpass" not in l and l.strip()]
            if lines:
                print("\n".join(lines), file=sys.stderr)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
