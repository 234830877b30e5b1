"""Accuracy measures shared by the tests (numpy, CPU).

These are the quality measures the tests gate on; none of them is part of
either solver.
"""
from __future__ import annotations

import numpy as np

U64 = np.finfo(np.float64).eps / 2  # unit roundoff


def herm_full(M: np.ndarray) -> np.ndarray:
    """Full Hermitian matrix from the upper triangle of M."""
    up = np.triu(M)
    full = up + np.triu(M, 1).conj().T
    np.fill_diagonal(full, np.real(np.diagonal(M)))
    return full


def backward_errors(H, S, w, C):
    """eta_i = ||H c - w S c|| / ((||H|| + |w| ||S||) ||c||) per column."""
    R = H @ C - (S @ C) * w[None, :]
    nh = np.linalg.norm(H, 2)
    ns = np.linalg.norm(S, 2)
    return np.linalg.norm(R, axis=0) / ((nh + np.abs(w) * ns) * np.linalg.norm(C, axis=0))


def s_orthonormality(S, C):
    k = C.shape[1]
    return np.abs(C.conj().T @ S @ C - np.eye(k)).max()


def subspace_agreement(S, C1, C2):
    """min over columns of |c1_i^H S c2_i| (1 for identical S-normalised
    eigenvectors up to a unit scalar)."""
    return np.abs(np.einsum("ij,ij->j", C1.conj(), S @ C2)).min()


def normalize_phase(C):
    """Scale each column so its largest-modulus entry (lowest index on
    ties) is real positive."""
    C = np.array(C, copy=True)
    idx = np.argmax(np.abs(C), axis=0)
    ph = C[idx, np.arange(C.shape[1])]
    return C * (np.abs(ph) / ph)[None, :]
