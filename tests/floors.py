"""The FP64 floor F of an input: how far the CPU oracle's own eigenvalues
move when H and S are perturbed at the unit roundoff.

Both the GPU path and the oracle are backward stable at best, so neither
can be expected to agree with the exact eigenvalues of the stored (H, S)
better than the spread that rounding-sized changes of the input produce.
F measures that spread with the oracle alone:

    F = max over draws, max over the k wanted i, |eps_i(H + dH, S + dS) - eps_i(H, S)| / |eps_i(H, S)|

with dH, dS random Hermitian of 2-norm u ||H||_2 and u ||S||_2 (u the FP64
unit roundoff).  The whole-solve tests gate each wanted eigenvalue's
relative error at max(1e-12, 10 F).  Stored floors (tests/golden/floors.json)
are written by tests/golden/make_floors.py, which calls only this module,
the oracle and the seeded input generators.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import oracle

U64 = np.finfo(np.float64).eps / 2
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "floors.json")


def oracle_eigenvalues(H: np.ndarray, S: np.ndarray) -> np.ndarray:
    """All n eigenvalues of H c = eps S c (ascending) by the oracle's route
    without eigenvectors: Cholesky, reduction by substitution, one-stage
    Householder tridiagonalisation, implicit QL."""
    U = oracle.cholesky(S)
    A = oracle.reduce(H, U)
    d, e, _, _ = oracle.tridiag(A)
    w, _ = oracle.tql(d, e, vectors=False)
    return w


def norm2_hermitian(M: np.ndarray) -> float:
    """||M||_2 of a Hermitian matrix (upper triangle read) by the oracle."""
    d, e, _, _ = oracle.tridiag(M)
    w, _ = oracle.tql(d, e, vectors=False)
    return float(np.abs(w).max())


def _random_hermitian(n: int, cplx: bool, rng: np.random.Generator) -> np.ndarray:
    g = rng.standard_normal((n, n))
    if cplx:
        g = (g + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
    return np.asfortranarray(0.5 * (g + g.conj().T))


def floor(H: np.ndarray, S: np.ndarray, k: int, seed: int = 0, draws: int = 2, w: np.ndarray | None = None,
          norm_h: float | None = None, norm_s: float | None = None, eig_fn=None) -> dict:
    """F (relative, over the k wanted) and its normwise companion
    max_i |d eps_i| / max |eps| (over all n) for one input.  eig_fn(H, S)
    gives the oracle's eigenvalues (default: the Cholesky route)."""
    n = H.shape[0]
    cplx = np.iscomplexobj(H) or np.iscomplexobj(S)
    eig_fn = oracle_eigenvalues if eig_fn is None else eig_fn
    w = eig_fn(H, S) if w is None else w
    nh = norm2_hermitian(H) if norm_h is None else norm_h
    ns = norm2_hermitian(S) if norm_s is None else norm_s
    rng = np.random.default_rng([seed, n, 7919])
    f_rel = 0.0
    f_nrm = 0.0
    for _ in range(draws):
        gh = _random_hermitian(n, cplx, rng)
        gs = _random_hermitian(n, cplx, rng)
        dh = gh * (U64 * nh / norm2_hermitian(gh))
        ds = gs * (U64 * ns / norm2_hermitian(gs))
        wp = eig_fn(H + dh, S + ds)
        if len(wp) != len(w):
            continue  # the perturbation moved a retained/omitted boundary: not a rounding spread
        dw = np.abs(wp - w)
        f_rel = max(f_rel, float((dw[:k] / np.maximum(np.abs(w[:k]), np.finfo(float).tiny)).max()))
        f_nrm = max(f_nrm, float(dw.max() / np.abs(w).max()))
    return {"F": f_rel, "F_normwise": f_nrm}


def key(kind: str, n: int, cplx: bool, sigma_min: float, seed: int, frac: float, extra: str = "") -> str:
    """Name of a stored floor: generator and its arguments."""
    s = "%s/n=%d/%s/smin=%g/seed=%d/f=%g" % (kind, n, "z" if cplx else "d", sigma_min, seed, frac)
    return s + ("/" + extra if extra else "")


_cache = None


def stored(k: str) -> dict:
    """The stored floor of a case; a case without one is an error (run
    tests/golden/make_floors.py)."""
    global _cache
    if _cache is None:
        with open(GOLDEN) as f:
            _cache = json.load(f)["floors"]
    if k not in _cache:
        raise KeyError("no stored floor for %s: run python tests/golden/make_floors.py" % k)
    return _cache[k]


def eig_gate(F: float) -> float:
    """Per-eigenvalue relative gate for an input with floor F."""
    return max(1e-12, 10.0 * F)


# normwise gate of the whole-solve tests: max |w - w_ref| / max |w_ref|
NORMWISE_GATE = 1e-11


def eig_errors(w: np.ndarray, w_ref: np.ndarray, k: int):
    """(max relative error over the k wanted, normwise error over all
    returned eigenvalues)."""
    m = min(len(w), len(w_ref))
    rel = np.abs(w[:k] - w_ref[:k]) / np.maximum(np.abs(w_ref[:k]), np.finfo(float).tiny)
    nrm = np.abs(w[:m] - w_ref[:m]).max() / np.abs(w_ref[:m]).max()
    return float(rel.max()), float(nrm)


def check_eigs(w: np.ndarray, w_ref: np.ndarray, k: int, fl: dict, label: str = "",
               normwise_gate: float | None = None) -> tuple:
    """Gate a whole solve's eigenvalues against the oracle's on the same
    input: each of the k wanted within max(1e-12, 10 F) relatively, and all
    returned ones within NORMWISE_GATE (or normwise_gate) of max |w_ref|.
    Prints the figures; returns (relative, normwise, relative gate)."""
    rel, nrm = eig_errors(w, w_ref, k)
    gate = eig_gate(fl["F"])
    print("%s eig rel %.2e (gate %.1e, F %.1e) normwise %.2e (floor %.1e)" %
          (label, rel, gate, fl["F"], nrm, fl["F_normwise"]), flush=True)
    assert rel <= gate, (label, rel, gate)
    assert nrm <= (NORMWISE_GATE if normwise_gate is None else normwise_gate), (label, nrm)
    return rel, nrm, gate
