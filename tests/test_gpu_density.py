"""Density matrix from the eigenvectors (gevd_density), against the oracle's
plain definition P_ij = sum_l f_l conj(c_li) c_lj and its energy-weighted
counterpart.  Elementwise gate: both sides sum k products per entry, so
each differs from the exact sum by at most k u (conj(|C|) F |C|^T)_ij; the
gate is twice that, entry by entry.  Invariants on the GPU result: P
Hermitian, sum_ij P_ij S_ij = sum_l f_l."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2502_02460_amd import synth
from tests.gpu_util import dev, host, log
from tests.linalg_checks import U64

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,cplx", [(1, False), (65, True), (300, False), (333, True), (700, True)])
def test_density_against_oracle(gpu_lib, n, cplx):
    p = synth.pencil(n, cplx, 1e-6, 3700 + n, 0.3)
    s = gpu_lib.Solver()
    w, C = s.solve(dev(p.H), dev(p.S), p.k)
    rng = np.random.default_rng(n)
    f = np.where(np.arange(p.k) < (2 * p.k) // 3, 2.0, rng.uniform(0.0, 2.0, p.k))  # filled, then fractional
    Pg, Qg = s.density(C, dev(f[:, None])[:, 0], w, energy_weighted=True)
    Pg, Qg, Ch, wh = host(Pg), host(Qg), host(C), host(w)
    s.close()
    P = oracle.density(Ch, f)
    Q = oracle.density(Ch, f, wh[: p.k])
    bP = 2 * p.k * U64 * ((np.abs(Ch) * f[None, :]) @ np.abs(Ch).T)
    bQ = 2 * p.k * U64 * ((np.abs(Ch) * np.abs(f * wh[: p.k])[None, :]) @ np.abs(Ch).T)
    eP = np.max(np.abs(Pg - P) / np.maximum(bP, np.finfo(float).tiny))
    eQ = np.max(np.abs(Qg - Q) / np.maximum(bQ, np.finfo(float).tiny))
    herm = np.abs(Pg - Pg.conj().T).max()
    count = float(np.real(np.sum(Pg * p.S)))
    log(f"density n={n} k={p.k} cplx={cplx}: |P - P_ref| / bound {eP:.2e}, Q {eQ:.2e}; "
        f"electrons {count:.12f} of {f.sum():.12f}")
    assert eP <= 1.0 and eQ <= 1.0
    assert herm == 0.0
    assert abs(count - f.sum()) < 1e-9 * f.sum()
