"""The pivot rule of the search kernels at the largest supported text
(n = 2^31 - 1, Section IV's (L + R) / 2 reading), compiled for the CPU with
the undefined-behaviour sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_midpoint_at_the_largest_text(tmp_path):
    exe = tmp_path / "pivot_check"
    src = os.path.join(ROOT, "tests", "native", "pivot_check.cpp")
    inc = os.path.join(ROOT, "paper_1303_3692_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                    f"-I{inc}", src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
