"""The C interface without a GPU: every function include/gevd.h declares is
exported by libgevd.so, and the host-side parts (argument validation before
any launch, error strings, workspace sizing) behave as documented."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gevd.h")
SO = os.path.join(ROOT, "paper_2502_02460_amd", "libgevd.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gevd_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(SO):
        pytest.skip("libgevd.so not built")
    return ctypes.CDLL(SO)


def test_header_declares_the_interface():
    names = declared()
    for must in ("gevd_create", "gevd_destroy", "gevd_solve", "gevd_cholesky", "gevd_invert_upper", "gevd_reduce",
                 "gevd_eigh", "gevd_backtransform", "gevd_stedc", "gevd_strerror", "gevd_workspace_bytes"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_null_handle_is_argument_one(lib):
    P, I = ctypes.c_void_p, ctypes.c_int
    lib.gevd_solve.argtypes = [P, I, I, I, P, I, P, I, P, P, I]
    assert lib.gevd_solve(None, 0, 4, 2, None, 4, None, 4, None, None, 4) == -1
    lib.gevd_cholesky.argtypes = [P, I, I, P, I]
    assert lib.gevd_cholesky(None, 0, 4, None, 4) == -1
    lib.gevd_stedc.argtypes = [P, I, I, P, P, P, P, I]
    assert lib.gevd_stedc(None, 4, 2, None, None, None, None, 4) == -1
    lib.gevd_create.argtypes = [P, I]
    assert lib.gevd_create(None, 0) == -1
    lib.gevd_solve_batched_noalloc.argtypes = [P, I, P, P]
    assert lib.gevd_solve_batched_noalloc(None, 1, None, None) == -1
    D = ctypes.c_double
    lib.gevd_solve_reduced.argtypes = [P, I, I, I, D, P, I, P, I, P, P, I, P, P]
    assert lib.gevd_solve_reduced(None, 0, 4, 2, 1e-5, None, 4, None, 4, None, None, 4, None, None) == -1
    lib.gevd_get_warnings.argtypes = [P, P]
    assert lib.gevd_get_warnings(None, None) == -1


def test_strerror_and_workspace(lib):
    lib.gevd_strerror.restype = ctypes.c_char_p
    lib.gevd_strerror.argtypes = [ctypes.c_int]
    assert lib.gevd_strerror(0) == b"success"
    assert b"positive definite" in lib.gevd_strerror(3)
    assert b"non-finite" in lib.gevd_strerror(-1001)
    lib.gevd_workspace_bytes.restype = ctypes.c_size_t
    lib.gevd_workspace_bytes.argtypes = [ctypes.c_int] * 3
    assert lib.gevd_workspace_bytes(0, 0, 1) == 0      # n < 1
    assert lib.gevd_workspace_bytes(0, 10, 11) == 0    # nev > n
    assert lib.gevd_workspace_bytes(2, 10, 5) == 0     # bad dtype
    small = lib.gevd_workspace_bytes(0, 256, 64)
    big = lib.gevd_workspace_bytes(1, 1024, 256)
    assert 0 < small < big
    # complex needs more than real at the same size
    assert lib.gevd_workspace_bytes(1, 512, 128) > lib.gevd_workspace_bytes(0, 512, 128)


def test_batched_entry_points_validate_on_host(lib):
    P, I = ctypes.c_void_p, ctypes.c_int
    lib.gevd_solve_batched.argtypes = [P, I, P, P]
    assert lib.gevd_solve_batched(None, 1, None, None) == -1
    lib.gevd_batch_create.argtypes = [P, I, P, P]
    assert lib.gevd_batch_create(None, 1, None, None) == -1
    lib.gevd_batch_run.argtypes = [P, P]
    assert lib.gevd_batch_run(None, None) == -1
    lib.gevd_batch_run_async.argtypes = [P, P]
    assert lib.gevd_batch_run_async(None, None) == -1
    lib.gevd_batch_destroy.argtypes = [P]
    assert lib.gevd_batch_destroy(None) == -1
    lib.gevd_set_batch_shape.argtypes = [P, I, I, I, I]
    assert lib.gevd_set_batch_shape(None, 0, 64, 256, 1) == -1
    lib.gevd_tune_batched.argtypes = [P, I, I, I, P, P]
    assert lib.gevd_tune_batched(None, 0, 64, 8, None, None) == -1
    lib.gevd_set_overlap.argtypes = [P, I, I, P, I]
    assert lib.gevd_set_overlap(None, 0, 4, None, 4) == -1


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
