"""AddressSanitizer and UndefinedBehaviorSanitizer runs of the host code (CPU).

  - the FP64 oracle (oracle/lbm_oracle.c), built with gcc and driven by
    tests/native/oracle_sanitized.c: every exported function on ragged
    lattices with rough walls, both collision operators, both electric-force
    directions, with leak detection;
  - the host side of liblbm (the library's sources with the sanitizers on the
    host compilation only; device code is compiled as usual and never
    launched), driven by tests/native/host_sanitized.cpp: workspace layouts,
    flag words, the per-row plain mask and the window of it the FP32 step
    kernel reads for every possible chunking, and the argument checks that
    run before the first HIP call.
Either driver exits non-zero on a sanitizer report or a failed check.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_0708_4182_amd", "csrc")
SOURCES = ["lbm_api.hip", "lbm_batch.hip", "lbm_kernels.hip", "net_api.hip", "net_kernels.hip"]

pytestmark = pytest.mark.slow


def run(cmd, env=None, timeout=600):
    res = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    out = res.stdout + res.stderr
    print(out[-4000:])
    return res.returncode, out


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    rc, _ = run([gcc, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer", "-ffp-contract=off", "-o", exe,
                 os.path.join(NATIVE, "oracle_sanitized.c"), "-lm"])
    assert rc == 0
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    rc, out = run([exe], env=env)
    assert rc == 0 and "oracle sanitizer run: ok" in out


def test_host_library_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "host_san")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    # sanitizers on the host compilation only
    flags += ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all"]
    rc, _ = run([hipcc, *flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", exe,
                 os.path.join(NATIVE, "host_sanitized.cpp"), *[os.path.join(CSRC, s) for s in SOURCES]])
    assert rc == 0
    # the HIP runtime's own allocations at exit are not this library's: no leak check
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    rc, out = run([exe], env=env)
    assert rc == 0 and "host sanitizer run: ok" in out
