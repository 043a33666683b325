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
