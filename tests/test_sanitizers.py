"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only,
no GPU is used):

* the oracle's C library, built with gcc -fsanitize=address,undefined and
  driven through every exported function on small inputs;
* libcouple's host side (argument checks, the device byte cap, couple_init
  without a device), built with the sanitizers on the host pass only and
  driven through every entry point with bad arguments.

Any sanitizer report aborts the driver (-fno-sanitize-recover=all).  Leak
checking is on for the oracle; for libcouple it is off, since the HIP runtime
keeps allocations of its own until exit.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")

pytestmark = pytest.mark.slow


def _run(cmd, env=None, cwd=None):
    return subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=cwd)


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "drv_oracle")
    b = _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", "-fopenmp", "-std=c99", os.path.join(HERE, "drv_oracle.c"),
              os.path.join(ROOT, "oracle", "coupling_oracle.c"), "-lm", "-o", exe])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    r = _run([exe], env=env)
    assert r.returncode == 0 and "oracle driver ok" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def _clangxx():
    for cand in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_library_host_paths_under_sanitizers(tmp_path):
    hipcc, clangxx = _hipcc(), _clangxx()
    if not hipcc or not clangxx:
        pytest.skip("hipcc / clang++ not available")
    lib = str(tmp_path / "libcouple_san.so")
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2602_15605_amd", "csrc", "*.hip")))
    # sanitizers on the host pass only: each -fsanitize= right after -Xarch_host
    b = _run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
              "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2602_15605_amd", "csrc"),
              "-o", lib] + srcs)
    assert b.returncode == 0, b.stderr[-4000:]
    exe = str(tmp_path / "drv_host")
    b = _run([clangxx, "-g", "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "drv_host.cpp"), lib,
              "-Wl,-rpath," + str(tmp_path), "-o", exe])
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    env.pop("COUPLE_MAX_DEVICE_BYTES", None)
    r = _run([exe], env=env)
    assert r.returncode == 0 and "host driver ok" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
