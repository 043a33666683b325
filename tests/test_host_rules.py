"""Host-only rules of the library checked with the system C++ compiler (no GPU,
no HIP): the book-keeping applied after every sweep path."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_13304_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_close_sweep_advances_every_handle_then_reports(tmp_path):
    exe = tmp_path / "close_sweep_check"
    src = os.path.join(ROOT, "tests", "host", "close_sweep_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC, src, "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_plan_compiler_under_address_and_undefined_sanitizers(tmp_path):
    """The plan compiler and geometry (host C++ only) built with
    AddressSanitizer and UndefinedBehaviorSanitizer: sweep and expectation
    plans of the hexagonal blocks N=2, 3, 4 and the 4x4-cell patch, every
    swallow order, T1 / T2, exact in-block contraction and the stability
    options, both parities; every reference starts inside its region."""
    exe = tmp_path / "plan_check"
    srcs = [os.path.join(ROOT, "tests", "host", "plan_check.cpp"),
            os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "geometry.cpp")]
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", "-I", CSRC, *srcs, "-o", str(exe)], check=True)
    env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               ASAN_OPTIONS="detect_leaks=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0, out.stdout[-4000:] + out.stderr[-4000:]
    assert out.stdout.strip().endswith("ok")
