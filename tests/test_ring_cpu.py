"""The launch-descriptor ring's placement arithmetic (host, CPU): built with
g++ from the library's own header and run over long sequences of puts."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2601_03086_amd", "csrc")


def test_ring_placement_stays_in_bounds(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "ring_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-I" + CSRC, os.path.join(HERE, "ring_check.cpp"),
                    "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stdout + r.stderr
