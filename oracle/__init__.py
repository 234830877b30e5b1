"""CPU oracle for the generalized eigenproblem H C = eps S C (paper Eq. (2)).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark may import this package.  The GPU solver does not
import it, and it does not import the GPU solver: the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, FP64, OpenMP over
independent rows/columns).  This module only marshals numpy arrays.  Every
matrix is passed column-major; complex matrices are complex128.

Functions follow the paper's steps (section "Solving the generalized
eigenproblem"): ``cholesky`` (step 1), ``reduce`` (steps 2-3, done by
substitution), ``tridiag`` + ``tql`` (the standard eigenproblem, one-stage
Householder then implicit QL), ``apply_q`` and ``backsub`` (the
back-transformation), and ``gevd`` for the whole solve.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

E_NONFINITE = -101
E_NOCONV = -102


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(_HERE, "oracle_core.inc"))):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_SO)
            P = ctypes.c_void_p
            I = ctypes.c_int
            D = ctypes.c_double
            for sfx in ("d", "z"):
                getattr(L, "oracle_cholesky_" + sfx).argtypes = [I, P, I]
                getattr(L, "oracle_reduce_" + sfx).argtypes = [I, P, I, P, I, P, I]
                getattr(L, "oracle_tridiag_" + sfx).argtypes = [I, P, I, P, P, P]
                getattr(L, "oracle_tridiag_" + sfx).restype = None
                getattr(L, "oracle_apply_q_" + sfx).argtypes = [I, I, P, I, P, P, I]
                getattr(L, "oracle_apply_q_" + sfx).restype = None
                getattr(L, "oracle_backsub_" + sfx).argtypes = [I, I, P, I, P, I]
                getattr(L, "oracle_backsub_" + sfx).restype = None
                getattr(L, "oracle_gevd_" + sfx).argtypes = [I, I, P, I, P, I, P, P, I, P]
            L.oracle_reduce_d.restype = None
            L.oracle_reduce_z.restype = None
            L.oracle_tql.argtypes = [I, P, P, P, I]
            L.oracle_sturm_count.argtypes = [I, P, P, D]
            L.oracle_threads.argtypes = []
            _lib = L
    return _lib


def _sfx(a: np.ndarray) -> str:
    return "z" if np.iscomplexobj(a) else "d"


def _f(a: np.ndarray, cplx: bool) -> np.ndarray:
    return np.asfortranarray(a, dtype=np.complex128 if cplx else np.float64)


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def threads() -> int:
    return int(lib().oracle_threads())


def cholesky(S: np.ndarray) -> np.ndarray:
    """Upper U with S = U^H U (only the upper triangle of S is read); the
    strictly lower part of the result is zero.  Raises on a non positive
    definite leading minor."""
    cplx = np.iscomplexobj(S)
    U = _f(S, cplx).copy(order="F")
    n = U.shape[0]
    info = getattr(lib(), "oracle_cholesky_" + _sfx(U))(n, _p(U), n)
    if info != 0:
        raise OracleError("S is not positive definite at leading minor %d" % info)
    return np.triu(U)


def reduce(H: np.ndarray, U: np.ndarray) -> np.ndarray:
    """A = U^{-H} H U^{-1} (upper triangles of H and U are read)."""
    cplx = np.iscomplexobj(H) or np.iscomplexobj(U)
    Hf, Uf = _f(H, cplx), _f(U, cplx)
    n = Hf.shape[0]
    A = np.zeros((n, n), dtype=Hf.dtype, order="F")
    getattr(lib(), "oracle_reduce_" + ("z" if cplx else "d"))(n, _p(Hf), n, _p(Uf), n, _p(A), n)
    return A


def tridiag(A: np.ndarray):
    """One-stage Householder tridiagonalisation.  Returns (d, e, refl, tau)
    where refl/tau encode Q (Q^H A Q = tridiag(d, e))."""
    cplx = np.iscomplexobj(A)
    R = _f(A, cplx).copy(order="F")
    n = R.shape[0]
    d = np.zeros(n)
    e = np.zeros(max(n, 1))
    tau = np.zeros(max(n, 1), dtype=R.dtype)
    getattr(lib(), "oracle_tridiag_" + _sfx(R))(n, _p(R), n, _p(d), _p(e), _p(tau))
    return d, e[: max(n - 1, 0)].copy(), R, tau


def apply_q(refl: np.ndarray, tau: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Q C for the Q encoded by (refl, tau) from ``tridiag``."""
    cplx = np.iscomplexobj(refl)
    Cf = _f(C, cplx).copy(order="F")
    n, k = Cf.shape
    getattr(lib(), "oracle_apply_q_" + _sfx(refl))(n, k, _p(refl), n, _p(np.ascontiguousarray(tau)), _p(Cf), n)
    return Cf


def backsub(U: np.ndarray, C: np.ndarray) -> np.ndarray:
    """U^{-1} C for upper triangular U."""
    cplx = np.iscomplexobj(U) or np.iscomplexobj(C)
    Uf = _f(U, cplx)
    Cf = _f(C, cplx).copy(order="F")
    n, k = Cf.shape
    getattr(lib(), "oracle_backsub_" + ("z" if cplx else "d"))(n, k, _p(Uf), n, _p(Cf), n)
    return Cf


def tql(d: np.ndarray, e: np.ndarray, vectors: bool = True):
    """Eigen-decomposition of the symmetric tridiagonal (d, e): returns
    (w ascending, Z or None)."""
    n = len(d)
    dd = np.array(d, dtype=np.float64)
    ee = np.zeros(max(n, 1))
    ee[: n - 1] = e[: n - 1]
    Z = np.zeros((n, n), order="F") if vectors else None
    info = lib().oracle_tql(n, _p(dd), _p(ee), _p(Z) if vectors else None, n)
    if info != 0:
        raise OracleError("implicit QL did not converge")
    return dd, Z


def sturm_count(d: np.ndarray, e: np.ndarray, x: float) -> int:
    """Number of eigenvalues of tridiag(d, e) strictly below x."""
    dd = np.ascontiguousarray(d, dtype=np.float64)
    ee = np.zeros(max(len(dd), 1))
    ee[: len(dd) - 1] = e[: len(dd) - 1]
    return int(lib().oracle_sturm_count(len(dd), _p(dd), _p(ee), float(x)))


def gevd(H: np.ndarray, S: np.ndarray, k: int | None = None):
    """Whole solve.  Returns (w: all n eigenvalues ascending, C: n x k
    S-orthonormal eigenvectors of the k smallest, times: 6 phase seconds
    [Cholesky, reduce, tridiag, solve, back(Q), back(U^-1)])."""
    cplx = np.iscomplexobj(H) or np.iscomplexobj(S)
    Hf, Sf = _f(H, cplx), _f(S, cplx)
    n = Hf.shape[0]
    k = n if k is None else k
    w = np.zeros(n)
    C = np.zeros((n, max(k, 1)), dtype=Hf.dtype, order="F")
    times = np.zeros(6)
    info = getattr(lib(), "oracle_gevd_" + ("z" if cplx else "d"))(
        n, k, _p(Hf), n, _p(Sf), n, _p(w), _p(C), n, _p(times))
    if info == E_NONFINITE:
        raise OracleError("non-finite input")
    if info == E_NOCONV:
        raise OracleError("tridiagonal QL did not converge")
    if info < 0:
        raise OracleError("argument %d invalid" % (-info))
    if info > 0:
        raise OracleError("S is not positive definite at leading minor %d" % info)
    return w, C, times


def _herm_from_upper(M: np.ndarray) -> np.ndarray:
    """Full Hermitian matrix from the upper triangle of M (the triangle the
    solver reads)."""
    up = np.triu(M, 1)
    full = up + up.conj().T
    full[np.diag_indices(M.shape[0])] = np.real(np.diagonal(M))
    return np.asfortranarray(full)


def eigh(A: np.ndarray, k: int | None = None):
    """Standard Hermitian eigenproblem A z = eps z (both triangles of the
    Hermitian A read): one-stage Householder tridiagonalisation, implicit QL
    with eigenvectors, back-transformation by the reflectors.  Returns (w:
    all n eigenvalues ascending, Z: n x k orthonormal eigenvectors of the k
    smallest)."""
    n = A.shape[0]
    k = n if k is None else k
    d, e, R, tau = tridiag(A)
    w, Z = tql(d, e, vectors=True)
    Zk = np.asfortranarray(Z[:, :k]).astype(R.dtype)
    return w, apply_q(R, tau, Zk)


def gevd_reduced(H: np.ndarray, S: np.ndarray, k: int, delta: float):
    """The route for an ill-conditioned overlap described at the end of the
    paper's section on reducing the generalized eigenproblem: S is
    diagonalised, S = D diag(sigma) D^H; the eigenvectors D_i whose sigma_i
    is below delta are omitted; in the basis X = D_r diag(sigma_r)^(-1/2) of
    the m retained ones the problem is the standard one
    (X^H H X) c~ = eps c~ (order m); and C = X c~, which is S-orthonormal.
    Upper triangles of H and S are read.

    Returns (w: the m eigenvalues of the reduced problem ascending, C: n x k
    eigenvectors of the k smallest, sigma: all n eigenvalues of S ascending,
    m).  Raises OracleError when fewer than k eigenvectors are retained."""
    Sf = _herm_from_upper(S)
    Hf = _herm_from_upper(H)
    n = Sf.shape[0]
    sigma, D = eigh(Sf, n)
    keep = sigma >= delta
    m = int(keep.sum())
    if m < k:
        raise OracleError("only %d overlap eigenvectors have sigma >= delta, fewer than k = %d" % (m, k))
    X = np.asfortranarray(D[:, keep] / np.sqrt(sigma[keep])[None, :])
    At = X.conj().T @ Hf @ X
    At = np.asfortranarray(0.5 * (At + At.conj().T))
    w, Z = eigh(At, k)
    C = np.asfortranarray(X @ Z)
    return w, C, sigma, m


def density(C: np.ndarray, f: np.ndarray, eps: np.ndarray | None = None) -> np.ndarray:
    """The paper's density matrix P_ij = sum_l f_l conj(c_li) c_lj (section on
    density-matrix based solutions), c_l the l-th eigenvector (column l of
    C), f_l its occupation number; with eps, the energy-weighted
    counterpart sum_l f_l eps_l conj(c_li) c_lj.  Written out as
    conj(C) diag(w) C^T with w = f (or f * eps)."""
    w = np.asarray(f, dtype=np.float64) * (1.0 if eps is None else np.asarray(eps, dtype=np.float64))
    return np.asfortranarray((np.conj(C) * w[None, :]) @ C.T)
