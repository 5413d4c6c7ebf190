"""Host code under the sanitizers (CPU only): the oracle with AddressSanitizer
and UndefinedBehaviorSanitizer, driven through every run mode; the host side of
the C ABI (validation, planning, workspace layout, batches, error strings,
checkpoint sizes) with AddressSanitizer and leak checking, linked against the
built kernels but touching no GPU.  Device code is never instrumented."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
PKG = os.path.join(ROOT, "paper_1105_4840_amd")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_main")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-o", exe, os.path.join(HERE, "oracle_main.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
    r = _run([exe], env=env, timeout=600)
    assert "done 0" in r.stdout


def _kernel_objects():
    import importlib.util
    spec = importlib.util.spec_from_file_location("ppp_pkg_build", os.path.join(PKG, "build.py"))
    build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(build)
    names = [f"shape_{t}_{g}x{b}.hip.o" for g, b in build.shapes() for t in ("float", "double")]
    names += [src + ".o" for src in build.SOURCES if src.endswith(".hip")]
    return [os.path.join(PKG, "_build", n) for n in names]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_host_runtime_under_address_sanitizer(tmp_path):
    objs = _kernel_objects()
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("kernel objects not built (run the package build first)")
    csrc = os.path.join(PKG, "csrc")
    flags = ["-x", "hip", "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
             "-I", os.path.join(ROOT, "include"), "-I", csrc]
    host = []
    for src in (os.path.join(csrc, "ppp_runtime.cpp"), os.path.join(csrc, "ppp_adaptive.cpp"),
                os.path.join(HERE, "runtime_main.cpp")):
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        _run(["hipcc", *flags, "-c", src, "-o", o])
        host.append(o)
    exe = str(tmp_path / "runtime_main")
    _run(["hipcc", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-o", exe, *host, *objs])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"), timeout=600)
    assert "done 0" in r.stdout
