"""Host-only parts of the served form, built with the system C++ compiler and
checked on the CPU:

* the device-phase gate (csrc/devgate.h), stressed by tests/devgate_check.cpp
  (three shared users, one exclusive user that never pauses): the two sides
  must never overlap, and neither may starve;
* the request-state allocator (csrc/arena.h), checked by
  tests/arena_check.cpp against a granule map: bounds, no overlap, first
  fit, the byte count in use, and coalescing back to one block.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2404_17101_amd", "csrc")


def _build_and_run(tmp_path, name, extra=()):
    exe = str(tmp_path / name)
    subprocess.run(["g++", "-O2", "-std=c++17", *extra, "-I", CSRC, os.path.join(HERE, name + ".cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    return subprocess.run([exe], capture_output=True, text=True, timeout=60)


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_device_phase_gate_excludes_and_alternates(tmp_path):
    r = _build_and_run(tmp_path, "devgate_check", ("-pthread",))
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_request_state_allocator_against_a_model(tmp_path):
    r = _build_and_run(tmp_path, "arena_check")
    assert r.returncode == 0, r.stdout + r.stderr
