"""Route selection of the persistent full -> band panel kernel, on the CPU.

Concurrent solves on one device must not run two persistent panel grids at
once (each needs all its workgroups resident together).  The library's
process-wide arbiter (csrc/arbiter.hpp, host-only C++) gives the persistent
route to one handle per device at a time and routes the others to one
launch per panel column; this compiles a small driver against that header
and checks the selection, nesting, per-device independence and mutual
exclusion under contention."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_panel_arbiter(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "arbiter_check")
    r = subprocess.run([cxx, "-std=c++17", "-O1", "-pthread", os.path.join(HERE, "arbiter_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
