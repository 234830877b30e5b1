"""Inputs of the whole-solve parity tests (shapes, seeds), shared by the
tests and by tests/golden/make_floors.py, which stores each input's FP64
floor.  Every input is a seeded draw of paper_2502_02460_amd.synth."""
from __future__ import annotations

from paper_2502_02460_amd import synth
from tests import floors

# test_gpu_stages.test_solve_parity: (n, wanted fraction, sigma_min), seed 800 + n
SOLVE = [(1, 1.0, 1e-3), (3, 1.0, 1e-3), (256, 1.0, 1e-3), (300, 0.3, 1e-6), (513, 0.25, 1e-6)]
# test_gpu_stages.test_band_width_tridiagonal_and_solve: (n, b), seed 1100 + n + b
# (b = 8 takes the single-wave bulge-chasing kernel, the others the workgroup one)
BANDS = [(129, 40), (300, 64), (700, 64), (333, 48), (201, 8)]
# test_gpu_stages.test_per_column_panel_route: n, seed 1500 + n
PER_COLUMN = [700, 1100]
# test_gpu_gemm_tiles: forced GEMM tile per process, (n, complex), seed 2100 + n
TILES = [(260, False), (260, True), (390, True)]
# test_gpu_batched: (n, complex, sigma_min, fraction), seed 4000 + index
BATCHED_MIX = [(1, False, 1e-3, 1.0), (2, True, 1e-3, 1.0), (7, False, 1e-3, 1.0), (64, True, 1e-6, 0.3),
               (65, False, 1e-6, 0.3), (128, False, 1e-3, 1.0), (130, True, 1e-6, 0.3), (256, True, 1e-6, 0.3),
               (257, False, 1e-6, 0.3), (512, False, 1e-6, 0.3), (512, True, 1e-6, 0.3), (333, True, 1e-3, 0.5)]
# test_gpu_resident: n, seed 900 + n, three SCF iterations
RESIDENT = [200, 600]
RESIDENT_ITERS = 3


def solve_pencil(n, frac, smin, cplx):
    return synth.pencil(n, cplx, smin, 800 + n, frac), floors.key("pencil", n, cplx, smin, 800 + n, frac)


def band_pencil(n, b, cplx):
    return (synth.pencil(n, cplx, 1e-6, 1100 + n + b, 0.3),
            floors.key("pencil", n, cplx, 1e-6, 1100 + n + b, 0.3))


def per_column_pencil(n, cplx):
    return synth.pencil(n, cplx, 1e-6, 1500 + n, 0.3), floors.key("pencil", n, cplx, 1e-6, 1500 + n, 0.3)


def tile_pencil(n, cplx):
    return synth.pencil(n, cplx, 1e-6, 2100 + n, 0.3), floors.key("pencil", n, cplx, 1e-6, 2100 + n, 0.3)


def batched_pencils():
    return [(synth.pencil(n, c, smin, 4000 + i, frac), floors.key("pencil", n, c, smin, 4000 + i, frac))
            for i, (n, c, smin, frac) in enumerate(BATCHED_MIX)]


def resident_inputs(n, cplx):
    """(pencil, [(H_t, floor key) for the SCF iterations])."""
    p = synth.pencil(n, cplx, 1e-6, 900 + n, 0.3)
    its = [(synth.scf_perturbation(p.H, request=n, it=it),
            floors.key("pencil", n, cplx, 1e-6, 900 + n, 0.3, "scf=%d" % it)) for it in range(RESIDENT_ITERS)]
    return p, its


def config_pencil(name):
    """A benchmark configuration at its full size, drawn on the CPU with
    pinned BLAS kernels (synth.pinned_problem: the same bits on any AVX2
    host)."""
    c = synth.CONFIGS[name]
    p, _ = synth.pinned_problem("pencil", c["n"], c["cplx"], c["sigma_min"], c["seed"], c["frac"])
    return p, floors.key("pencil", c["n"], c["cplx"], c["sigma_min"], c["seed"], c["frac"])


def all_cases(include_large: bool = True):
    """(key, H, S, k, ||H||_2, ||S||_2) of every stored-floor case."""
    out = []

    def add(p, key, H=None):
        out.append((key, p.H if H is None else H, p.S, p.k, None if H is not None else float(abs(p.lam).max()),
                    float(abs(p.sigma).max())))

    for cplx in (False, True):
        for n, frac, smin in SOLVE:
            add(*solve_pencil(n, frac, smin, cplx))
        for n, b in BANDS:
            add(*band_pencil(n, b, cplx))
        for n in PER_COLUMN:
            add(*per_column_pencil(n, cplx))
        for n in RESIDENT:
            p, its = resident_inputs(n, cplx)
            for H, key in its:
                add(p, key, H)
    for n, cplx in TILES:
        add(*tile_pencil(n, cplx))
    for p, key in batched_pencils():
        add(p, key)
    if include_large:
        add(*config_pencil("c1"))
    return out
