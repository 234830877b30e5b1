"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something other than itself: a closed
form, an exact rational computation, a mathematical invariant, or LAPACK
(scipy) as an independent library route.  Together they are chosen so that
a dropped term, a wrong sign, a wrong index or a transposed/unconjugated
operand in any oracle stage fails at least one test.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from paper_2502_02460_amd import synth
from tests.linalg_checks import U64, backward_errors, s_orthonormality

RNG = np.random.default_rng(1234)


# ---------------------------------------------------------------- Cholesky
@pytest.mark.parametrize("cplx", [False, True])
def test_cholesky_identity_and_diagonal(cplx):
    n = 37
    dt = np.complex128 if cplx else np.float64
    U = oracle.cholesky(np.eye(n, dtype=dt))
    assert np.array_equal(U, np.eye(n))
    dg = RNG.uniform(0.5, 9.0, n)
    U = oracle.cholesky(np.diag(dg).astype(dt))
    assert np.allclose(U, np.diag(np.sqrt(dg)), rtol=0, atol=4 * U64 * 3)


def test_cholesky_2x2_closed_form():
    # S = [[a, b], [conj(b), c]] -> U = [[sqrt(a), b/sqrt(a)], [0, sqrt(c - |b|^2/a)]]
    a, b, c = 4.0, 1.5 - 2.0j, 9.0
    U = oracle.cholesky(np.array([[a, b], [np.conj(b), c]]))
    expect = np.array([[2.0, b / 2.0], [0.0, math.sqrt(c - abs(b) ** 2 / a)]])
    assert np.allclose(U, expect, rtol=4 * U64, atol=0)


@pytest.mark.parametrize("cplx", [False, True])
def test_cholesky_reconstructs_and_ignores_lower(cplx):
    p = synth.pencil(96, cplx, 1e-3, 11)
    S = p.S.copy(order="F")
    S[np.tril_indices(96, -1)] = np.nan  # the lower triangle must never be read
    U = oracle.cholesky(S)
    assert np.all(np.real(np.diagonal(U)) > 0) and np.all(np.imag(np.diagonal(U)) == 0)
    err = np.abs(U.conj().T @ U - p.S).max() / np.abs(p.S).max()
    assert err < 96 * U64 * 8
    # the factor of a PD matrix is unique: LAPACK's upper factor must agree
    Ul = sl.cholesky(p.S, lower=False)
    assert np.abs(U - Ul).max() / np.abs(Ul).max() < 1e-12


def test_cholesky_not_pd_reports_minor():
    S = np.diag([1.0, 2.0, 3.0, -1.0, 5.0])
    with pytest.raises(oracle.OracleError, match="minor 4"):
        oracle.cholesky(S)


# ---------------------------------------------------------------- reduction
@pytest.mark.parametrize("cplx", [False, True])
def test_reduce_inverts_the_congruence(cplx):
    p = synth.pencil(80, cplx, 1e-4, 12)
    U = oracle.cholesky(p.S)
    H = p.H.copy(order="F")
    H[np.tril_indices(80, -1)] = np.nan  # lower triangle of H must be ignored
    A = oracle.reduce(H, U)
    assert np.array_equal(A, A.conj().T)
    back = U.conj().T @ A @ U
    assert np.abs(back - p.H).max() / np.abs(p.H).max() < 1e-12
    # the same congruence through an explicit inverse (independent route)
    Ui = sl.solve_triangular(U, np.eye(80, dtype=U.dtype), lower=False)
    A2 = Ui.conj().T @ p.H @ Ui
    assert np.abs(A - A2).max() / np.abs(A2).max() < 1e-10


# ---------------------------------------------------------------- tridiagonal
def test_tql_toeplitz_closed_form():
    # tridiag(b, a, b): eigenvalues a + 2 b cos(j pi/(n+1)), eigenvectors
    # sqrt(2/(n+1)) sin(i j pi/(n+1)).
    for n, a, b in [(1, 0.3, 1.0), (2, 0.0, 1.0), (50, 0.0, 1.0), (257, -1.5, 0.75)]:
        w, Z = oracle.tql(np.full(n, a), np.full(max(n - 1, 0), b))
        j = np.arange(1, n + 1)
        exact = np.sort(a + 2 * b * np.cos(j * np.pi / (n + 1)))
        assert np.abs(w - exact).max() <= 8 * n * U64 * (abs(a) + 2 * abs(b))
        i = np.arange(1, n + 1)[:, None]
        X = math.sqrt(2.0 / (n + 1)) * np.sin(i * j[None, :] * np.pi / (n + 1))
        order = np.argsort(a + 2 * b * np.cos(j * np.pi / (n + 1)))
        X = X[:, order]
        overlap = np.abs(np.sum(X * Z, axis=0))
        assert np.all(overlap > 1 - 1e-10)


def test_tql_diagonal_and_sturm():
    d = RNG.standard_normal(40)
    w, Z = oracle.tql(d, np.zeros(39))
    assert np.array_equal(w, np.sort(d))
    assert np.array_equal(np.abs(Z), np.abs(Z).round())  # a permutation
    # Sturm counts of a random tridiagonal at midpoints of its eigenvalues
    d = RNG.standard_normal(300)
    e = RNG.standard_normal(299)
    w, _ = oracle.tql(d, e, vectors=False)
    mids = 0.5 * (w[1:] + w[:-1])
    for i, x in enumerate(mids):
        assert oracle.sturm_count(d, e, x) == i + 1
    assert oracle.sturm_count(d, e, w[0] - 1.0) == 0
    assert oracle.sturm_count(d, e, w[-1] + 1.0) == 300


def test_tql_against_lapack_tridiagonal():
    d = RNG.standard_normal(500)
    e = RNG.standard_normal(499)
    w, Z = oracle.tql(d, e)
    wl = sl.eigh_tridiagonal(d, e, eigvals_only=True)
    assert np.abs(w - wl).max() < 500 * U64 * 8
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.abs(T @ Z - Z * w[None, :]).max() < 1e-12
    assert np.abs(Z.T @ Z - np.eye(500)).max() < 1e-12


@pytest.mark.parametrize("cplx", [False, True])
def test_householder_tridiagonalisation(cplx):
    n = 70
    p = synth.pencil(n, cplx, 1e-2, 13)
    A = oracle.reduce(p.H, oracle.cholesky(p.S))
    d, e, refl, tau = oracle.tridiag(A)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    Q = oracle.apply_q(refl, tau, np.eye(n, dtype=A.dtype))
    nrm = np.abs(A).max()
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-13
    assert np.abs(Q.conj().T @ A @ Q - T).max() / nrm < 1e-13
    assert np.all(np.isreal(e))


# ---------------------------------------------------------------- full solve
@pytest.mark.parametrize("cplx", [False, True])
def test_gevd_2x2_quadratic(cplx):
    for _ in range(20):
        h = RNG.standard_normal(4)
        s = RNG.standard_normal(4)
        h12 = h[2] + (1j * h[3] if cplx else 0.0)
        s12 = 0.3 * (s[2] + (1j * s[3] if cplx else 0.0))
        H = np.array([[h[0], h12], [np.conj(h12), h[1]]])
        S = np.array([[1.0 + abs(s[0]), s12], [np.conj(s12), 1.0 + abs(s[1])]])
        a = S[0, 0].real * S[1, 1].real - abs(s12) ** 2
        b = -(H[0, 0].real * S[1, 1].real + H[1, 1].real * S[0, 0].real - 2 * (h12 * np.conj(s12)).real)
        c = H[0, 0].real * H[1, 1].real - abs(h12) ** 2
        disc = math.sqrt(b * b - 4 * a * c)
        roots = np.sort([(-b - disc) / (2 * a), (-b + disc) / (2 * a)])
        w, C, _ = oracle.gevd(H, S, 2)
        assert np.abs(w - roots).max() <= 1e-13 * max(1.0, np.abs(roots).max())
        assert s_orthonormality(S, C) < 1e-14


@pytest.mark.parametrize("cplx", [False, True])
def test_gevd_commuting_pencil_exact(cplx):
    n = 120
    p = synth.commuting_pencil(n, cplx, 1e-5, 21)
    w, C, _ = oracle.gevd(p.H, p.S, n)
    # eps_i = lam_i / sigma_i exactly.  The Cholesky route is normwise
    # backward stable on the standard form A = U^-H H U^-1, so every
    # eigenvalue carries an absolute error of order n u ||A|| with
    # ||A|| = max |eps| (about 2.6e6 here); 1e-10 relative to ||A|| leaves a
    # margin of ~10x over what was observed and is 7 orders below the effect
    # of any dropped term or wrong sign.
    scale = np.abs(p.exact).max()
    assert np.abs(w - p.exact).max() / scale < 1e-10
    assert s_orthonormality(p.S, C) < 1e-10


@pytest.mark.parametrize("cplx", [False, True])
def test_gevd_identity_overlap_and_scalar_pencil(cplx):
    n = 90
    p = synth.identity_overlap(n, cplx, 22)
    w, C, _ = oracle.gevd(p.H, p.S, 30)
    assert np.abs(w - p.exact).max() < 64 * n * U64 * 50
    # H = alpha S: one n-fold eigenvalue alpha; C must still be S-orthonormal
    q = synth.pencil(n, cplx, 1e-3, 23)
    alpha = -2.75
    w, C, _ = oracle.gevd(alpha * q.S, q.S, n)
    assert np.abs(w - alpha).max() < 1e-11
    assert s_orthonormality(q.S, C) < 1e-11


@pytest.mark.parametrize("cplx", [False, True])
def test_gevd_invariants_c0_shape(cplx):
    c = synth.CONFIGS["c0"]
    p = synth.pencil(c["n"], cplx, c["sigma_min"], c["seed"])
    n = c["n"]
    w, C, times = oracle.gevd(p.H, p.S, n)
    assert np.all(np.diff(w) >= 0)
    assert backward_errors(p.H, p.S, w, C).max() < 1e-13
    assert s_orthonormality(p.S, C) < 1e-12
    # trace of the standard form equals the eigenvalue sum
    A = oracle.reduce(p.H, oracle.cholesky(p.S))
    assert abs(np.sum(w) - np.trace(A).real) < 1e-11 * np.abs(w).sum()
    # Sylvester inertia of H - x S (LDL^T with pivoting, LAPACK) at points
    # between consecutive eigenvalues gives the eigenvalue count below x
    for kk in (1, 13, n // 2, n - 1):
        x = 0.5 * (w[kk - 1] + w[kk])
        _, D, _ = sl.ldl(p.H - x * p.S, hermitian=True)
        neg = int(np.sum(np.linalg.eigvalsh(D) < 0))
        assert neg == kk
    assert len(times) == 6 and np.all(times >= 0)


@pytest.mark.parametrize("cplx", [False, True])
def test_gevd_against_lapack(cplx):
    n = 300
    p = synth.pencil(n, cplx, 1e-6, 24, 0.3)
    w, C, _ = oracle.gevd(p.H, p.S, p.k)
    wl, Cl = sl.eigh(p.H, p.S)
    scale = np.abs(wl).max()
    # two independent FP64 routes at kappa(S) = 1e6 differ by a few 1e-12
    # normwise (the conditioning of the reduction, not of either code)
    assert np.abs(w - wl).max() / scale < 1e-10
    # eigenvectors agree up to a unit scalar (spectrum is simple here)
    gap = np.min(np.diff(wl[: p.k + 1])) / scale
    assert gap > 1e-9
    ov = np.abs(np.einsum("ij,ij->j", C.conj(), p.S @ Cl[:, : p.k]))
    assert ov.min() > 1 - 1e-6


def test_gevd_argument_and_input_errors():
    H = np.eye(3)
    with pytest.raises(oracle.OracleError, match="argument"):
        oracle.gevd(H, H, 0)
    with pytest.raises(oracle.OracleError, match="argument"):
        oracle.gevd(H, H, 4)
    Hn = H.copy()
    Hn[0, 2] = np.nan
    with pytest.raises(oracle.OracleError, match="non-finite"):
        oracle.gevd(Hn, H, 2)
    S = np.diag([1.0, -1.0, 1.0])
    with pytest.raises(oracle.OracleError, match="minor 2"):
        oracle.gevd(H, S, 2)


# ----------------------------------------------- exact rational brute force
def _herm_rand_int(n, cplx, rng, lo=-4, hi=5):
    M = [[None] * n for _ in range(n)]
    for i in range(n):
        for j in range(i, n):
            re = int(rng.integers(lo, hi))
            im = int(rng.integers(lo, hi)) if (cplx and i != j) else 0
            M[i][j] = (Fraction(re), Fraction(im))
            M[j][i] = (Fraction(re), Fraction(-im))
    return M


def _neg_pivots(H, S, x):
    """Exact inertia count of H - x S by LDL^H in rational arithmetic
    (complex numbers as (re, im) Fraction pairs).  Returns None when an
    exact zero pivot appears (x hits an eigenvalue of a leading block)."""
    n = len(H)
    A = [[(H[i][j][0] - x * S[i][j][0], H[i][j][1] - x * S[i][j][1]) for j in range(n)] for i in range(n)]
    neg = 0
    for k in range(n):
        p = A[k][k][0]
        if p == 0:
            return None
        if p < 0:
            neg += 1
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                # A[i][j] -= A[i][k] * A[k][j] / p
                ar, ai = A[i][k]
                br, bi = A[k][j]
                pr = (ar * br - ai * bi) / p
                pi = (ar * bi + ai * br) / p
                A[i][j] = (A[i][j][0] - pr, A[i][j][1] - pi)
    return neg


def _count_below(H, S, x):
    c = _neg_pivots(H, S, x)
    eps = Fraction(1, 10 ** 40)
    while c is None:
        x += eps
        c = _neg_pivots(H, S, x)
    return c


def _exact_eigs(H, S, tol=Fraction(1, 10 ** 28)):
    n = len(H)
    lo, hi = Fraction(-10 ** 6), Fraction(10 ** 6)
    out = []
    for k in range(1, n + 1):
        a, b = lo, hi  # count_below(a) < k <= count_below(b)
        while b - a > tol:
            m = (a + b) / 2
            if _count_below(H, S, m) >= k:
                b = m
            else:
                a = m
        out.append((a + b) / 2)
    return out


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [3, 5])
def test_gevd_brute_force_rational(cplx, n):
    rng = np.random.default_rng(100 + n + 7 * cplx)
    H = _herm_rand_int(n, cplx, rng)
    B = _herm_rand_int(n, cplx, rng, -2, 3)
    # S = B^H B + 2 I: rational, Hermitian positive definite
    S = [[None] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            re = sum(B[l][i][0] * B[l][j][0] + B[l][i][1] * B[l][j][1] for l in range(n))
            im = sum(B[l][i][0] * B[l][j][1] - B[l][i][1] * B[l][j][0] for l in range(n))
            S[i][j] = (re + (2 if i == j else 0), im)
    exact = np.array([float(v) for v in _exact_eigs(H, S)])
    to_np = lambda M: np.array([[float(a) + 1j * float(b) for (a, b) in row] for row in M])
    Hn, Sn = to_np(H), to_np(S)
    if not cplx:
        Hn, Sn = Hn.real.copy(), Sn.real.copy()
    w, C, _ = oracle.gevd(Hn, Sn, n)
    assert np.abs(w - exact).max() <= 1e-13 * max(1.0, np.abs(exact).max())
    assert backward_errors(Hn, Sn, w, C).max() < 1e-14


# ------------------------------------------- ill-conditioned overlap route
@pytest.mark.parametrize("cplx", [False, True])
def test_eigh_standard_against_closed_form_and_lapack(cplx):
    # tridiag(1, 0, 1) embedded by a Haar similarity has eigenvalues 2 cos(j pi/(n+1))
    n = 70
    rng = np.random.default_rng(31)
    Q = synth.haar(n, rng, cplx)
    T = np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    A = np.asfortranarray(Q @ T @ Q.conj().T)
    A = np.asfortranarray(0.5 * (A + A.conj().T))
    w, Z = oracle.eigh(A, 20)
    exact = np.sort(2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    assert np.abs(w - exact).max() < 64 * n * U64
    assert np.abs(A @ Z - Z * w[None, :20]).max() < 64 * n * U64
    assert np.abs(Z.conj().T @ Z - np.eye(20)).max() < 64 * n * U64
    assert np.abs(w - sl.eigvalsh(A)).max() < 64 * n * U64


@pytest.mark.parametrize("cplx", [False, True])
def test_reduced_route_commuting_closed_form(cplx):
    """H = V diag(lam) V^H, S = V diag(sigma) V^H with some sigma below delta:
    the retained basis spans exactly the V columns with sigma >= delta, so the
    reduced eigenvalues are lam_i / sigma_i over those, and nothing else."""
    n, delta = 96, 1e-5
    rng = np.random.default_rng(41)
    V = synth.haar(n, rng, cplx)
    sigma = np.exp(rng.uniform(np.log(1e-9), 0.0, n))
    sigma[:10] = np.exp(rng.uniform(np.log(1e-12), np.log(1e-7), 10))  # surely dropped
    lam = synth.core_like_spectrum(n, rng)
    S = np.asfortranarray(0.5 * ((V * sigma) @ V.conj().T + ((V * sigma) @ V.conj().T).conj().T))
    H = np.asfortranarray(0.5 * ((V * lam) @ V.conj().T + ((V * lam) @ V.conj().T).conj().T))
    keep = sigma >= delta
    order = np.argsort(lam[keep] / sigma[keep])
    exact = (lam[keep] / sigma[keep])[order]
    sig_of = sigma[keep][order]
    k = 25
    w, C, sig, m = oracle.gevd_reduced(H, S, k, delta)
    assert m == int(keep.sum())
    assert np.abs(np.sort(sig) - np.sort(sigma)).max() < 64 * n * U64
    # Rounding errors of order n u ||.|| in H, S and in S's eigenvectors move
    # eps_i = lam_i/sigma_i, to first order, by (||dH|| + |eps_i| ||dS||)
    # ||c_i||^2 with ||c_i||^2 = 1/sigma_i; the standard solve of the reduced
    # matrix (norm max |eps|) adds n u max |eps|.  Each retained eigenvalue
    # is held to 8 n u ((||H|| + |eps_i| ||S||) / sigma_i + max |eps|):
    # condition-limited by 1/delta, not by 1/sigma_min = 1e12 as the
    # Cholesky route would be.  A wrong scaling of the basis or a dropped
    # term moves them by O(|eps_i|).
    bound = 8 * n * U64 * ((np.abs(lam).max() + np.abs(exact) * sigma.max()) / sig_of + np.abs(exact).max())
    assert np.all(np.abs(w - exact) <= bound)
    assert s_orthonormality(S, C) < 1e-10
    # every column is an exact eigenpair of the commuting pencil
    assert backward_errors(H, S, w[:k], C).max() < 1e-12


@pytest.mark.parametrize("cplx", [False, True])
def test_reduced_route_without_dropping_equals_the_cholesky_route(cplx):
    """delta below every sigma_i: nothing is omitted, X spans the whole
    space, and the eigenvalues are those of H c = eps S c."""
    p = synth.pencil(80, cplx, 1e-3, 43, 0.4)
    w_ref, C_ref, _ = oracle.gevd(p.H, p.S, p.k)
    w, C, _, m = oracle.gevd_reduced(p.H, p.S, p.k, 1e-9)
    assert m == 80
    assert np.abs(w - w_ref).max() / np.abs(w_ref).max() < 1e-12
    assert np.abs(np.abs(np.einsum("ij,ij->j", C.conj(), p.S @ C_ref)) - 1.0).max() < 1e-9


@pytest.mark.parametrize("cplx", [False, True])
def test_reduced_route_galerkin_condition(cplx):
    """For a generic pencil with dropped directions, each returned pair
    satisfies the Galerkin condition in the retained basis:
    X^H (H c - eps S c) = 0; and C^H S C = I."""
    p = synth.pencil(90, cplx, 1e-8, 47, 0.3)
    delta = 1e-5
    w, C, sig, m = oracle.gevd_reduced(p.H, p.S, p.k, delta)
    assert m == int((sig >= delta).sum()) and m < 90
    Sf = p.S
    sigma, D = oracle.eigh(Sf, 90)
    X = D[:, sigma >= delta] / np.sqrt(sigma[sigma >= delta])[None, :]
    R = X.conj().T @ (p.H @ C - (Sf @ C) * w[None, : p.k])
    scale = np.abs(w[: p.k]).max()
    assert np.abs(R).max() / scale < 1e-11
    assert s_orthonormality(Sf, C) < 1e-11


def test_reduced_route_rank_error():
    p = synth.pencil(30, False, 1e-8, 49, 1.0)
    with pytest.raises(oracle.OracleError):
        oracle.gevd_reduced(p.H, p.S, 30, 1e-5)


# ------------------------------------------------------------ density matrix
@pytest.mark.parametrize("cplx", [False, True])
def test_density_brute_force_and_invariants(cplx):
    """P_ij = sum_l f_l conj(c_li) c_lj written as three nested loops at a tiny
    order; with S-orthonormal eigenvectors: sum_ij P_ij S_ij = sum_l f_l
    (the electron count), P Hermitian, and with every state filled
    (k = n, f = 1) P = conj(S^-1)."""
    p = synth.pencil(7, cplx, 1e-2, 53, 1.0)
    w, C, _ = oracle.gevd(p.H, p.S, 7)
    rng = np.random.default_rng(55)
    f = rng.uniform(0.0, 2.0, 5)
    P = oracle.density(C[:, :5], f)
    Pb = np.zeros((7, 7), dtype=C.dtype)
    for i in range(7):
        for j in range(7):
            for l in range(5):
                Pb[i, j] += f[l] * np.conj(C[i, l]) * C[j, l]
    assert np.abs(P - Pb).max() < 1e-13 * np.abs(Pb).max()
    assert np.abs(P - P.conj().T).max() < 1e-13 * np.abs(P).max()
    assert abs(np.sum(P * p.S) - f.sum()) < 1e-11 * f.sum()
    Pall = oracle.density(C, np.ones(7))
    assert np.abs(Pall @ np.conj(p.S) - np.eye(7)).max() < 1e-10
    Q = oracle.density(C[:, :5], f, w[:5])
    assert abs(np.sum(Q * p.S) - np.sum(f * w[:5])) < 1e-11 * np.abs(f * w[:5]).sum()
