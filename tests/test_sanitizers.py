"""AddressSanitizer and UndefinedBehaviorSanitizer builds (CPU only).

1. The FP64 oracle with the input generator, built with gcc and both
   sanitizers (and LeakSanitizer), runs a small problem through every oracle
   entry point.
2. The library with its host code instrumented (device code unchanged: the
   sanitizers apply to the host pass only) runs the host runtime's layout path
   -- repacking into the compact and the general records, the index checks,
   the super-voxel schedules -- and the load call's argument checks, without
   a device (tests/sanitize/layout_driver.cpp).
Any report of either sanitizer fails the run.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-4000:] + r.stderr[-4000:]
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "san_oracle")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-fopenmp", "-std=c11", "-D_DEFAULT_SOURCE",
          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "mace_oracle.c"),
          os.path.join(ROOT, "mace_inputs", "sysmat.c"), "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", OMP_NUM_THREADS="4")
    out = _run([exe], env=env)
    assert out.strip().endswith("OK"), out


@pytest.mark.slow
def test_host_runtime_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_1911_09278_amd", "csrc")
    srcs = sorted(f for f in os.listdir(csrc) if f.endswith((".cpp", ".hip")))
    flags = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-mllvm", "-pragma-unroll-threshold=1000000",
             "-I", os.path.join(ROOT, "include")] + SAN_HOST

    def comp(f):
        o = str(tmp_path / (f + ".o"))
        _run([HIPCC] + flags + ["-x", "hip", "-c", os.path.join(csrc, f), "-o", o])
        return o

    with ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 4))) as ex:
        objs = list(ex.map(comp, srcs))
    gen = str(tmp_path / "sysmat.o")
    _run(["gcc", "-O1", "-g", "-c", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC",
          os.path.join(ROOT, "mace_inputs", "sysmat.c"), "-o", gen])
    drv = str(tmp_path / "driver.o")
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include")] + SAN_HOST +
         ["-c", os.path.join(ROOT, "tests", "sanitize", "layout_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "san_layout")
    _run([HIPCC, "--offload-arch=gfx950"] + SAN_HOST + objs + [gen, drv, "-o", exe, "-lpthread"])
    # the HIP runtime keeps allocations for the process lifetime: leaks are
    # not reported, every other finding is fatal
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    out = _run([exe], env=env)
    assert out.strip().endswith("OK"), out
