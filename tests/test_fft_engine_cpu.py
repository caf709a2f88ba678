"""The library's LDS FFT engine run on the CPU (thread per lane, real barriers)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_line_fft_engine_on_cpu(tmp_path):
    exe = tmp_path / "fft_lines"
    src = os.path.join(HERE, "cpu_harness", "fft_lines.cpp")
    r = subprocess.run(["g++", "-std=c++20", "-O1", "-pthread", "-I" + os.path.join(HERE, "cpu_harness"),
                        src, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
