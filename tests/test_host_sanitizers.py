"""The host library under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The host sources (DAG build, schedulers, memory model, planner, C ABI) are
compiled with g++ and -fsanitize=address,undefined (every report fatal) into
one program with tests/sanitize/driver.cpp, which drives every host entry
point on seeded DAGs and on malformed input; the device runtime is replaced by
tests/sanitize/device_stub.cpp.  Any memory error, leak or undefined behaviour
fails the run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_02257_amd", "csrc")
HOST = ["host/dag.cpp", "host/sched.cpp", "host/plan.cpp", "host/kplan.cpp", "capi.cpp"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_library_is_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "driver"
    srcs = [os.path.join(CSRC, s) for s in HOST] + [
        os.path.join(ROOT, "tests", "sanitize", "device_stub.cpp"),
        os.path.join(ROOT, "tests", "sanitize", "driver.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, "-I", os.path.join(ROOT, "include"), *srcs, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "sanitizer driver: ok" in r.stdout
