"""The one-stage Householder tridiagonalisation (GEVD_OPT_STAGES = 1), the
route the paper ran on GPUs for full spectra, against the oracle's own
one-stage tridiagonalisation and whole solve.

Stage: the tridiagonal's eigenvalues (oracle QL on the GPU's d, e) against
the oracle's tridiagonal of the same A, normwise max(64 n, 4096) u.  Whole
solves: each wanted eigenvalue within max(1e-12, 10 F) of the oracle's (F
the input's floor, tests/floors.py), all within 1e-11 normwise; backward
error <= 1e-11; S-orthonormality within max(1e-11, 10x the oracle's);
all n pairs (k = n) at the c0 shape; panel edges and ragged tails."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2502_02460_amd import synth
from tests import cases, floors
from tests.gpu_util import dev, host, log
from tests.linalg_checks import U64, backward_errors, s_orthonormality

pytestmark = pytest.mark.gpu


def tol_eig(n):
    return max(64 * n, 4096) * U64


@pytest.fixture(scope="module")
def solver1(gpu_lib):
    s = gpu_lib.Solver(stages=1)
    yield s
    s.close()


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [1, 2, 3, 32, 33, 129, 300, 700])
def test_onestage_tridiagonal_spectrum(solver1, n, cplx):
    p = synth.pencil(n, cplx, 1e-2, 5600 + n)
    A0 = oracle.reduce(p.H, oracle.cholesky(p.S))
    d, e = solver1.tridiagonalize(dev(A0))
    d, e = host(d), host(e)
    w, _ = oracle.tql(d, e, vectors=False)
    dr, er, _, _ = oracle.tridiag(A0)
    w_ref, _ = oracle.tql(dr, er, vectors=False)
    err = np.abs(w - w_ref).max() / np.abs(w_ref).max()
    log(f"one-stage tridiagonal n={n} cplx={cplx}: eig diff {err:.2e}")
    assert err < tol_eig(n)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [2, 64, 300])
def test_onestage_eigh(solver1, n, cplx):
    p = synth.pencil(n, cplx, 1e-2, 5700 + n)
    A0 = oracle.reduce(p.H, oracle.cholesky(p.S))
    nev = max(1, int(0.3 * n))
    w, Z = solver1.eigh(dev(A0), nev)
    w, Z = host(w), host(Z)
    dr, er, _, _ = oracle.tridiag(A0)
    w_ref, _ = oracle.tql(dr, er, vectors=False)
    nrm = np.abs(w_ref).max()
    err = np.abs(w - w_ref).max() / nrm
    res = np.abs(A0 @ Z - Z * w[None, :nev]).max() / nrm
    orth = np.abs(Z.conj().T @ Z - np.eye(nev)).max()
    log(f"one-stage eigh n={n} cplx={cplx}: eig {err:.2e} res {res:.2e} orth {orth:.2e}")
    assert err < tol_eig(n) and res < tol_eig(n) and orth < 1e-11


def _whole(s, p, key, label, fl=None):
    w_ref, C_ref, _ = oracle.gevd(p.H, p.S, p.k)
    w, C = s.solve(dev(p.H), dev(p.S), p.k)
    w, C = host(w), host(C)
    floors.check_eigs(w, w_ref, p.k, fl if fl is not None else floors.stored(key), label)
    eta = backward_errors(p.H, p.S, w[: p.k], C).max()
    orth, orth_ref = s_orthonormality(p.S, C), s_orthonormality(p.S, C_ref)
    log(f"  eta {eta:.2e} orth {orth:.2e} (oracle {orth_ref:.2e})")
    assert eta < 1e-11
    assert orth < max(1e-11, 10 * orth_ref)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,frac,smin", cases.SOLVE)
def test_onestage_solve_parity(solver1, n, frac, smin, cplx):
    p, key = cases.solve_pencil(n, frac, smin, cplx)
    _whole(solver1, p, key, f"one-stage solve n={n} k={p.k} cplx={cplx}:")


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", cases.PER_COLUMN)
def test_onestage_solve_larger(solver1, n, cplx):
    p, key = cases.per_column_pencil(n, cplx)
    _whole(solver1, p, key, f"one-stage solve n={n} k={p.k} cplx={cplx}:")


def test_onestage_all_pairs_c0_shape(solver1):
    c = synth.CONFIGS["c0"]
    p = synth.pencil(c["n"], c["cplx"], c["sigma_min"], c["seed"], c["frac"])
    _whole(solver1, p, None, f"one-stage c0 shape n={c['n']} all pairs:", fl=floors.floor(p.H, p.S, p.k))
