"""Host sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer), run on the CPU.

* The oracle: ``mpr_oracle.c`` built with gcc and both sanitizers, driven by ``sanitize/oracle_checks.c`` through
  every entry point and simulation mode on small and degenerate grids.
* The library's host code: every HIP source built with the sanitizers on the host pass only (the device code is
  built as usual), linked with ``sanitize/abi_host_checks.cpp``, which runs the workspace queries (including the
  batched rule over 300 scenes) and the argument checks that refuse a call before anything is enqueued.  No call
  reaches a GPU.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2212_01317_amd", "csrc")
SAN_HOST = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "mpr_oracle.c"),
                           os.path.join(HERE, "sanitize", "oracle_checks.c"), "-lm", "-o", exe])
    res = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "oracle sanitizer checks ok" in res.stdout


@pytest.mark.slow
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    import sys
    sys.path.insert(0, ROOT)
    from paper_2212_01317_amd.build import SOURCES
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", *SAN_HOST.split(), "-ffp-contract=off",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(HERE, "sanitize", "abi_host_checks.cpp")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([hipcc, *common, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "abi_host_checks")
    r = subprocess.run([hipcc, *SAN_HOST.split(), *objs, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    res = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "host ABI sanitizer checks ok" in res.stdout
