"""GPU parity tests, stage by stage, against the CPU oracle (through the C
interface).  Sizes span several 64-wide tiles and ragged tails.

Tolerances.  Stage tests of the standard problem: both routes are normwise
backward stable, so their eigenvalues differ by a multiple of n u ||A|| (u
the FP64 unit roundoff) and are compared as |w - w_ref| <= TOL_EIG *
max|w_ref|; factors elementwise relative to their largest entry.  Whole
generalized solves: each of the k wanted eigenvalues within max(1e-12, 10 F)
relatively of the oracle's, F the input's FP64 floor (tests/floors.py,
stored by tests/golden/make_floors.py), and all n within 1e-11 of max|w_ref|;
eigenvectors by backward error (<= 1e-11) and S-orthonormality.
"""
from __future__ import annotations

import numpy as np
import torch
import pytest
import scipy.linalg as sl

import oracle
from paper_2502_02460_amd import synth
from tests import cases, floors
from tests.gpu_util import dev, host, log
from tests.linalg_checks import U64, backward_errors, s_orthonormality

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 7, 64, 65, 200, 333]


def tol_eig(n):
    return max(64 * n, 4096) * U64


@pytest.fixture(scope="module")
def solver(gpu_lib):
    s = gpu_lib.Solver()
    yield s
    s.close()


# ----------------------------------------------------------------- step 1
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", SIZES)
def test_cholesky_parity(solver, n, cplx):
    p = synth.pencil(n, cplx, 1e-3, 100 + n)
    U_ref = oracle.cholesky(p.S)
    S = dev(p.S)
    solver.cholesky(S)
    U = np.triu(host(S))
    err = np.abs(U - U_ref).max() / np.abs(U_ref).max()
    log(f"cholesky n={n} cplx={cplx}: max rel diff {err:.2e}")
    assert err < 1e-12
    assert np.all(np.imag(np.diagonal(U)) == 0)


def test_cholesky_not_pd(solver, gpu_lib):
    for n, bad in [(10, 4), (150, 97)]:
        d = np.linspace(1, 2, n)
        d[bad - 1] = -1.0
        S = dev(np.diag(d))
        with pytest.raises(gpu_lib.NotPositiveDefinite) as ei:
            solver.cholesky(S)
        assert ei.value.code == bad


# ----------------------------------------------------------------- step 2
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", SIZES)
def test_invert_parity(solver, n, cplx):
    p = synth.pencil(n, cplx, 1e-3, 200 + n)
    U = oracle.cholesky(p.S)
    Ui_ref = oracle.backsub(U, np.eye(n, dtype=U.dtype))
    Ud = dev(U + np.tril(np.full((n, n), 7.0), -1))  # garbage below: must be ignored
    Ui = host(solver.invert_upper(Ud))
    assert np.all(Ui[np.tril_indices(n, -1)] == 0)
    err = np.abs(Ui - Ui_ref).max() / np.abs(Ui_ref).max()
    log(f"invert n={n} cplx={cplx}: max rel diff {err:.2e}")
    assert err < 1e-12


# ----------------------------------------------------------------- step 3
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", SIZES)
def test_reduce_parity(solver, n, cplx):
    p = synth.pencil(n, cplx, 1e-3, 300 + n)
    U = oracle.cholesky(p.S)
    A_ref = oracle.reduce(p.H, U)
    Ui = oracle.backsub(U, np.eye(n, dtype=U.dtype))
    H = p.H.copy(order="F")
    H[np.tril_indices(n, -1)] = np.nan  # only the upper triangle is read
    A = host(solver.reduce(dev(H), dev(Ui)))
    err = np.abs(A - A_ref).max() / np.abs(A_ref).max()
    log(f"reduce n={n} cplx={cplx}: max rel diff {err:.2e}")
    assert err < 1e-12
    assert np.abs(A - A.conj().T).max() == 0


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,nev", [(1, 1), (65, 20), (200, 61), (333, 333)])
def test_backtransform_parity(solver, n, nev, cplx):
    p = synth.pencil(n, cplx, 1e-3, 400 + n)
    U = oracle.cholesky(p.S)
    Ui = oracle.backsub(U, np.eye(n, dtype=U.dtype))
    rng = np.random.default_rng(n)
    Ct = rng.standard_normal((n, nev)) + (1j * rng.standard_normal((n, nev)) if cplx else 0)
    C_ref = oracle.backsub(U, Ct)
    C = host(solver.backtransform(dev(Ui), dev(Ct)))
    err = np.abs(C - C_ref).max() / np.abs(C_ref).max()
    log(f"backtransform n={n} nev={nev} cplx={cplx}: max rel diff {err:.2e}")
    assert err < 1e-12


# --------------------------------------------------------- tridiagonal D&C
def _tridiag_cases():
    rng = np.random.default_rng(5)
    out = []
    for n in (1, 2, 5, 33, 100, 300, 1000):
        out.append(("random", rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))))
    for n in (64, 257):
        out.append(("toeplitz", np.zeros(n), np.ones(n - 1)))
        dd = np.ones(n)
        dd[::3] = 2.0
        out.append(("clusters", dd, 1e-3 * np.ones(n - 1)))
        ee = rng.standard_normal(n - 1)
        ee[::7] = 0.0
        out.append(("split", rng.standard_normal(n), ee))
        m = (n - 1) // 2
        out.append(("wilkinson", np.abs(np.arange(-m, n - m)).astype(float), np.ones(n - 1)))
        out.append(("near-diag", np.ones(n), 1e-10 * rng.standard_normal(n - 1)))
    return out


@pytest.mark.parametrize("case", _tridiag_cases(), ids=lambda c: f"{c[0]}-{len(c[1])}")
def test_stedc_parity(solver, case):
    name, d, e = case
    n = len(d)
    nev = max(1, (3 * n) // 4)
    w_ref, Z_ref = oracle.tql(d, e)
    w, Z = solver.stedc(dev(d[:, None])[:, 0], dev(e[:, None])[:, 0] if n > 1 else dev(np.zeros((1, 1)))[:, 0], nev)
    w, Z = host(w), host(Z)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    nrm = max(np.abs(w_ref).max(), 1e-300)
    err = np.abs(w - w_ref).max() / nrm
    res = np.abs(T @ Z - Z * w[None, :nev]).max() / nrm
    orth = np.abs(Z.T @ Z - np.eye(nev)).max()
    log(f"stedc {name} n={n}: eig {err:.2e} res {res:.2e} orth {orth:.2e}")
    assert err < tol_eig(n)
    assert res < tol_eig(n)
    assert orth < 1e-12


# ------------------------------------------------------ reduction stages
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [2, 3, 40, 129, 300])
def test_band_spectrum(solver, n, cplx):
    p = synth.pencil(n, cplx, 1e-2, 500 + n)
    A0 = oracle.reduce(p.H, oracle.cholesky(p.S))
    b = solver.band_width(n, A0.dtype)
    Bd = host(solver.band(dev(A0)))
    B = np.zeros((n, n), dtype=A0.dtype)
    for r in range(b + 1):
        idx = np.arange(n - r)
        B[idx + r, idx] = Bd[r, : n - r]
    B = B + np.tril(B, -1).conj().T
    w_ref = sl.eigvalsh(A0)
    err = np.abs(sl.eigvalsh(B) - w_ref).max() / np.abs(w_ref).max()
    log(f"band n={n} b={b} cplx={cplx}: eig diff {err:.2e}")
    assert err < tol_eig(n)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [1, 2, 3, 40, 129, 300])
def test_tridiagonalize_spectrum(solver, n, cplx):
    p = synth.pencil(n, cplx, 1e-2, 600 + n)
    A0 = oracle.reduce(p.H, oracle.cholesky(p.S))
    d, e = solver.tridiagonalize(dev(A0))
    d, e = host(d), host(e)
    w, _ = oracle.tql(d, e, vectors=False)
    dr, er, _, _ = oracle.tridiag(A0)
    w_ref, _ = oracle.tql(dr, er, vectors=False)
    err = np.abs(w - w_ref).max() / np.abs(w_ref).max()
    log(f"tridiagonalize n={n} cplx={cplx}: eig diff {err:.2e}")
    assert err < tol_eig(n)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [1, 2, 5, 64, 129, 300])
def test_eigh_parity(solver, n, cplx):
    p = synth.pencil(n, cplx, 1e-2, 700 + n)
    A0 = oracle.reduce(p.H, oracle.cholesky(p.S))
    nev = max(1, int(0.3 * n))
    w, Z = solver.eigh(dev(A0), nev)
    w, Z = host(w), host(Z)
    dr, er, refl, tau = oracle.tridiag(A0)
    w_ref, _ = oracle.tql(dr, er, vectors=False)
    nrm = np.abs(w_ref).max()
    err = np.abs(w - w_ref).max() / nrm
    res = np.abs(A0 @ Z - Z * w[None, :nev]).max() / nrm
    orth = np.abs(Z.conj().T @ Z - np.eye(nev)).max()
    log(f"eigh n={n} cplx={cplx}: eig {err:.2e} res {res:.2e} orth {orth:.2e}")
    assert err < tol_eig(n)
    assert res < tol_eig(n)
    assert orth < 1e-11


# --------------------------------------------------------------- whole solve
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,frac,smin", cases.SOLVE)
def test_solve_parity(solver, n, frac, smin, cplx):
    p, key = cases.solve_pencil(n, frac, smin, cplx)
    w_ref, C_ref, _ = oracle.gevd(p.H, p.S, p.k)
    w, C = solver.solve(dev(p.H), dev(p.S), p.k)
    w, C = host(w), host(C)
    floors.check_eigs(w, w_ref, p.k, floors.stored(key), f"solve n={n} k={p.k} cplx={cplx} smin={smin}:")
    eta = backward_errors(p.H, p.S, w[: p.k], C).max()
    orth = s_orthonormality(p.S, C)
    orth_ref = s_orthonormality(p.S, C_ref)
    log(f"  eta {eta:.2e} orth {orth:.2e} (oracle orth {orth_ref:.2e})")
    assert eta < 1e-11
    assert orth < max(1e-11, 10 * orth_ref)


# ------------------------- band widths (single-wave and workgroup bulge chasing)
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,b", cases.BANDS)
def test_band_width_tridiagonal_and_solve(gpu_lib, n, b, cplx):
    s = gpu_lib.Solver(band=b)
    assert s.band_width(n, torch.complex128 if cplx else torch.float64) == b
    p, key = cases.band_pencil(n, b, cplx)
    A0 = oracle.reduce(p.H, oracle.cholesky(p.S))
    d, e = s.tridiagonalize(dev(A0))
    d, e = host(d), host(e)
    w, _ = oracle.tql(d, e, vectors=False)
    dr, er, _, _ = oracle.tridiag(A0)
    w_tri, _ = oracle.tql(dr, er, vectors=False)
    err_t = np.abs(w - w_tri).max() / np.abs(w_tri).max()
    w_ref, C_ref, _ = oracle.gevd(p.H, p.S, p.k)
    ws, C = s.solve(dev(p.H), dev(p.S), p.k)
    ws, C = host(ws), host(C)
    floors.check_eigs(ws, w_ref, p.k, floors.stored(key), f"band n={n} b={b} cplx={cplx}:")
    eta = backward_errors(p.H, p.S, ws[: p.k], C).max()
    orth, orth_ref = s_orthonormality(p.S, C), s_orthonormality(p.S, C_ref)
    log(f"  tridiag eig {err_t:.2e}; eta {eta:.2e} orth {orth:.2e} (oracle {orth_ref:.2e})")
    assert err_t < tol_eig(n)
    assert eta < 1e-11
    assert orth < max(1e-11, 10 * orth_ref)
    s.close()


# ------------------------------------- per-column panels (GEVD_OPT_PANEL = 0)
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", cases.PER_COLUMN)
def test_per_column_panel_route(gpu_lib, n, cplx):
    """The full -> band panels as one launch per column (the route for
    several solves sharing the device) give a solve of the same quality as
    the persistent panel kernel."""
    s = gpu_lib.Solver(persistent_panel=False)
    p, key = cases.per_column_pencil(n, cplx)
    w_ref, C_ref, _ = oracle.gevd(p.H, p.S, p.k)
    ws, C = s.solve(dev(p.H), dev(p.S), p.k)
    ws, C = host(ws), host(C)
    floors.check_eigs(ws, w_ref, p.k, floors.stored(key), f"per-column panels n={n} cplx={cplx}:")
    eta = backward_errors(p.H, p.S, ws[: p.k], C).max()
    orth, orth_ref = s_orthonormality(p.S, C), s_orthonormality(p.S, C_ref)
    log(f"  eta {eta:.2e} orth {orth:.2e} (oracle {orth_ref:.2e})")
    assert eta < 1e-11
    assert orth < max(1e-11, 10 * orth_ref)
    L = gpu_lib.load()
    assert L.gevd_set_option(s._h, gpu_lib.OPT_PANEL, 1) == 0
    assert L.gevd_set_option(s._h, gpu_lib.OPT_PANEL, 2) == -3
    s.close()
