"""The served form's device-phase gate (csrc/devgate.h) on the host: built
with the system C++ compiler and stressed by tests/devgate_check.cpp (three
shared users, one exclusive user that never pauses). The two sides must never
overlap, and neither may starve."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2404_17101_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_device_phase_gate_excludes_and_alternates(tmp_path):
    exe = str(tmp_path / "devgate_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-I", CSRC, os.path.join(HERE, "devgate_check.cpp"),
                    "-o", exe], check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
