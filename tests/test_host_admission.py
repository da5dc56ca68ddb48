"""Host-only checks of the request server's admission policy (gwc::Admission,
the FIFO-by-footprint scheduler of gwc_server.hip) on a fake executor: a small
C++ driver built with the address + undefined-behaviour sanitizers and with
the thread sanitizer, run on the CPU (no device)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "admission_driver.cpp")
INC = os.path.join(ROOT, "paper_2412_17132_amd", "csrc")


@pytest.mark.parametrize("sanitizer", ["address,undefined", "thread"])
def test_admission_policy_under_sanitizers(tmp_path, sanitizer):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "admission")
    build = subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                            f"-fsanitize={sanitizer}", "-pthread", "-I", INC, SRC, "-o", exe],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=180, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all checks passed" in run.stdout
