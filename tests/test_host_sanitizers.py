"""The library's host setup code (host_setup.cpp, spatial.cpp) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and run over small problems by
tests/host/sanitize_driver.cpp (no GPU, no HIP): any out-of-bounds access, use after free, leak,
signed overflow or misaligned access aborts the test program.  It also checks what the host code
computes: finite results, the weighted-form mass stencil against the Kronecker-assembled one, the
time factors against H_i, and the lane slots of every time-solve plan."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2311_18461_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_setup_under_sanitizers(tmp_path):
    exe = tmp_path / "sanitize_driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(HERE, "host", "sanitize_driver.cpp"), os.path.join(CSRC, "host_setup.cpp"),
           os.path.join(CSRC, "spatial.cpp"), "-o", str(exe)]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout[-2000:])
    assert run.returncode == 0, (run.stdout + run.stderr)[-6000:]
    assert "address sanitizer: on" in run.stdout and "OK (0 failed checks)" in run.stdout
