"""Every matrix-product tile against the oracle.

The tile of a product is chosen from its shape: the eight-wave tiles (real
128 x 128, and the complex 64 x 128 / 128 x 64 tiles in the three-product
form) only once a product has enough tiles to fill the device, i.e. at
orders far beyond what the oracle checks quickly.  GEVD_OPT_GEMM_TILE forces
one tile on every product of a handle's solve, so each tile runs the whole
generalized solve (Cholesky updates, inversion, both reduction products,
full -> band, the back-transformations, the divide-and-conquer merges) at
small order and is held to the whole-solve gates: each wanted eigenvalue
within max(1e-12, 10 F) of the oracle's (F the input's FP64 floor), all
within 1e-11 normwise, backward error <= 1e-11, S-orthonormality within
max(1e-11, 10x the oracle's).  One case also forces the b = 64 band that
the default picks from n = 4096 on."""
from __future__ import annotations

import functools

import pytest

import oracle
from tests import cases, floors
from tests.gpu_util import dev, host, log
from tests.linalg_checks import backward_errors, s_orthonormality

pytestmark = pytest.mark.gpu

# tiles the shape rule can pick (gemm.hip pick_tile): 0 = 64x64, 4 = 64x32,
# 5 = 32x64 (four waves); 6 = 128x128 (real), 7 = 128x64, 8 = 64x128 (eight
# waves; three-product form for complex)
REAL_TILES = [0, 4, 5, 6, 7, 8]
CPLX_TILES = [0, 4, 5, 7, 8]
PARAMS = ([(t, n, c) for n, c in cases.TILES if not c for t in REAL_TILES] +
          [(t, n, c) for n, c in cases.TILES if c for t in CPLX_TILES])


@functools.lru_cache(maxsize=None)
def _reference(n, cplx):
    p, key = cases.tile_pencil(n, cplx)
    w_ref, C_ref, _ = oracle.gevd(p.H, p.S, p.k)
    return p, key, w_ref, s_orthonormality(p.S, C_ref)


def _check(s, n, cplx, label):
    p, key, w_ref, orth_ref = _reference(n, cplx)
    w, C = s.solve(dev(p.H), dev(p.S), p.k)
    w, C = host(w), host(C)
    floors.check_eigs(w, w_ref, p.k, floors.stored(key), label)
    eta = backward_errors(p.H, p.S, w[: p.k], C).max()
    orth = s_orthonormality(p.S, C)
    log(f"  eta {eta:.2e} orth {orth:.2e} (oracle {orth_ref:.2e})")
    assert eta < 1e-11
    assert orth < max(1e-11, 10 * orth_ref)


@pytest.mark.parametrize("tile,n,cplx", PARAMS, ids=[f"tile{t}-n{n}-{'z' if c else 'd'}" for t, n, c in PARAMS])
def test_forced_tile_solve(gpu_lib, tile, n, cplx):
    s = gpu_lib.Solver(gemm_tile=tile)
    try:
        _check(s, n, cplx, f"tile {tile} n={n} cplx={cplx}:")
    finally:
        s.close()


def test_forced_tile_with_wide_band(gpu_lib):
    """Complex three-product tile with the b = 64 band of the large orders."""
    s = gpu_lib.Solver(gemm_tile=8, band=64)
    try:
        _check(s, 390, True, "tile 8, b = 64, n=390 complex:")
    finally:
        s.close()


def test_tile_option_validated(gpu_lib):
    s = gpu_lib.Solver()
    L = gpu_lib.load()
    assert L.gevd_set_option(s._h, gpu_lib.OPT_GEMM_TILE, 9) == -3
    assert L.gevd_set_option(s._h, gpu_lib.OPT_GEMM_TILE, -2) == -3
    assert L.gevd_set_option(s._h, gpu_lib.OPT_GEMM_TILE, -1) == 0
    s.close()
