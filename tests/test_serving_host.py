"""The tied-beam server's scheduler on the host, against a simulated device.

Compiles tests/serve_sched_test.cpp with the scheduler sources using g++
(once plain, once with AddressSanitizer and UndefinedBehaviorSanitizer) and
runs it.  No GPU and no HIP runtime are involved.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_08591_amd", "csrc")


@pytest.mark.parametrize("flags", [["-O2"], ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]],
                         ids=["plain", "asan_ubsan"])
def test_scheduler_host(flags):
    gxx = shutil.which("g++")
    assert gxx, "g++ is needed for the host scheduler test"
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "serve_sched_test")
        cmd = [gxx, "-std=c++17", "-Wall", "-Wextra", *flags, "-I", CSRC,
               os.path.join(ROOT, "tests", "serve_sched_test.cpp"), os.path.join(CSRC, "serve_sched.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "ALL OK" in r.stdout
