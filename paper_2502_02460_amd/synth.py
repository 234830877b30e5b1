"""Seeded synthetic inputs for the generalized eigenproblem H c = eps S c.

This module only draws random matrices.  It holds none of the solver's
arithmetic, and it is the one piece of code that both the CPU oracle's
tests and the GPU path's tests and benchmark use.

The paper's own matrices (FHI-aims Hamiltonian/overlap pairs, and the
N = 40960 matrix of its Table 1) are not available, so DFT-shaped stand-ins
are drawn instead:

* S = V diag(sigma) V^H with V Haar-random (orthogonal or unitary) and
  sigma log-uniform in [sigma_min, 1]; S is positive definite with
  condition number about 1/sigma_min, inside the range the paper allows
  (section "Solving the generalized eigenproblem": condition number of S
  well below about 1e12).
* H = W diag(lambda) W^H with an independent Haar W; 10 % of lambda
  (rounded) uniform in [-50, -5] (core-like states), the rest uniform in
  [-1, 3].
* Both are made exactly Hermitian as (M + M^H)/2 after the products.

Haar matrices come from the QR factorisation of a Gaussian matrix with the
diagonal-phase correction (Mezzadri, Notices AMS 54, 2007).

All matrices are returned in column-major (Fortran) order, the layout the
solver's C interface takes.  numpy is used for sizes the CPU handles in
seconds; ``*_torch`` variants draw large inputs directly in device memory.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Problem:
    """One generalized eigenproblem instance (column-major arrays)."""

    H: np.ndarray
    S: np.ndarray
    k: int
    lam: np.ndarray  # spectrum used for H
    sigma: np.ndarray  # spectrum used for S
    exact: np.ndarray | None = None  # known generalized eigenvalues, if any


def wanted(n: int, frac: float) -> int:
    """k = ceil(frac * n), at least 1."""
    return max(1, min(n, int(math.ceil(frac * n - 1e-9))))


def haar(n: int, rng: np.random.Generator, cplx: bool) -> np.ndarray:
    g = rng.standard_normal((n, n))
    if cplx:
        g = (g + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
    q, r = np.linalg.qr(g)
    dg = np.diagonal(r)
    ph = dg / np.abs(dg)
    return q * ph[None, :]


def core_like_spectrum(n: int, rng: np.random.Generator) -> np.ndarray:
    ncore = int(round(0.1 * n))
    lam = np.concatenate([rng.uniform(-50.0, -5.0, ncore), rng.uniform(-1.0, 3.0, n - ncore)])
    return lam


def log_uniform(n: int, lo: float, rng: np.random.Generator) -> np.ndarray:
    return np.exp(rng.uniform(math.log(lo), 0.0, n))


def _herm(m: np.ndarray) -> np.ndarray:
    return np.asfortranarray(0.5 * (m + m.conj().T))


def _from_spectrum(q: np.ndarray, vals: np.ndarray) -> np.ndarray:
    return _herm((q * vals[None, :]) @ q.conj().T)


def pencil(n: int, cplx: bool, sigma_min: float, seed: int, frac: float = 1.0) -> Problem:
    """The DFT-shaped pencil: independent Haar eigenbases for H and S."""
    rng = np.random.default_rng(seed)
    v = haar(n, rng, cplx)
    w = haar(n, rng, cplx)
    sigma = log_uniform(n, sigma_min, rng)
    lam = core_like_spectrum(n, rng)
    return Problem(H=_from_spectrum(w, lam), S=_from_spectrum(v, sigma), k=wanted(n, frac), lam=lam, sigma=sigma)


def commuting_pencil(n: int, cplx: bool, sigma_min: float, seed: int, frac: float = 1.0) -> Problem:
    """H = V diag(lam) V^H and S = V diag(sigma) V^H with the same V, so the
    generalized eigenvalues are exactly lam_i / sigma_i."""
    rng = np.random.default_rng(seed)
    v = haar(n, rng, cplx)
    sigma = log_uniform(n, sigma_min, rng)
    lam = core_like_spectrum(n, rng)
    return Problem(H=_from_spectrum(v, lam), S=_from_spectrum(v, sigma), k=wanted(n, frac), lam=lam,
                   sigma=sigma, exact=np.sort(lam / sigma))


def identity_overlap(n: int, cplx: bool, seed: int, frac: float = 1.0) -> Problem:
    """S = I: the generalized eigenvalues are the drawn lam exactly."""
    rng = np.random.default_rng(seed)
    w = haar(n, rng, cplx)
    lam = core_like_spectrum(n, rng)
    S = np.asfortranarray(np.eye(n, dtype=np.complex128 if cplx else np.float64))
    return Problem(H=_from_spectrum(w, lam), S=S, k=wanted(n, frac), lam=lam, sigma=np.ones(n),
                   exact=np.sort(lam))


def scf_perturbation(H0: np.ndarray, request: int, it: int, base_seed: int = 4) -> np.ndarray:
    """H_t = H_0 + 1e-3 (G + G^H)/2 with G iid N(0,1) (complex: N(0,1/2) +
    i N(0,1/2)), seeded by (request, iteration); not cumulative."""
    n = H0.shape[0]
    rng = np.random.default_rng([base_seed, request, it])
    g = rng.standard_normal((n, n))
    if np.iscomplexobj(H0):
        g = (g + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
    return np.asfortranarray(H0 + 1e-3 * 0.5 * (g + g.conj().T))


# The benchmark workloads (sizes, types and spectra), seeds 0..3: real n = 256
# (all pairs), real n = 4096 and 8192 (lowest 30 %), complex n = 16384 (lowest 25 %).
CONFIGS = {
    "c0": dict(n=256, cplx=False, sigma_min=1e-3, frac=1.0, seed=0),
    "c1": dict(n=4096, cplx=False, sigma_min=1e-6, frac=0.30, seed=1),
    "c2": dict(n=16384, cplx=True, sigma_min=1e-6, frac=0.25, seed=2),
    "c3": dict(n=8192, cplx=False, sigma_min=1e-6, frac=0.30, seed=3),
}


def config_problem(name: str) -> Problem:
    c = CONFIGS[name]
    return pencil(c["n"], c["cplx"], c["sigma_min"], c["seed"], c["frac"])


# ---------------------------------------------------------------------------
# Device-side generation for sizes numpy cannot produce in minutes.
# ---------------------------------------------------------------------------

def haar_torch(n: int, gen, cplx: bool, device):
    import torch

    dt = torch.complex128 if cplx else torch.float64
    if cplx:
        g = torch.randn(n, n, dtype=torch.float64, device=device, generator=gen) + 1j * torch.randn(
            n, n, dtype=torch.float64, device=device, generator=gen)
        g = g / math.sqrt(2.0)
    else:
        g = torch.randn(n, n, dtype=dt, device=device, generator=gen)
    q, r = torch.linalg.qr(g)
    dg = torch.diagonal(r)
    ph = dg / dg.abs()
    return q * ph[None, :]


def pencil_torch(n: int, cplx: bool, sigma_min: float, seed: int, frac: float, device, commuting: bool = False,
                 spectra: bool = False):
    """Same recipe as ``pencil`` drawn in device memory.  Returns (H, S, k,
    exact) where H and S are column-major views (stride (1, n)) and exact is
    the sorted lam/sigma for a commuting pencil, else None; with spectra=True
    also the drawn lam and sigma (so ||H||_2 = max |lam|, ||S||_2 = max sigma)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    v = haar_torch(n, gen, cplx, device)
    w = v if commuting else haar_torch(n, gen, cplx, device)
    u = torch.rand(n, dtype=torch.float64, device=device, generator=gen)
    sigma = torch.exp(u * math.log(sigma_min))
    ncore = int(round(0.1 * n))
    lam = torch.cat([
        -50.0 + 45.0 * torch.rand(ncore, dtype=torch.float64, device=device, generator=gen),
        -1.0 + 4.0 * torch.rand(n - ncore, dtype=torch.float64, device=device, generator=gen)])

    def build(q, vals):
        m = (q * vals.to(q.dtype)[None, :]) @ q.conj().T.contiguous()
        m = 0.5 * (m + m.conj().T)
        # column-major storage: the transpose of a contiguous tensor
        return m.T.contiguous().T

    H = build(w, lam)
    del w
    S = build(v, sigma)
    del v
    exact = torch.sort(lam / sigma).values if commuting else None
    if spectra:
        return H, S, wanted(n, frac), exact, lam, sigma
    return H, S, wanted(n, frac), exact


# ---------------------------------------------------------------------------
# Reproducible CPU draws.  numpy's QR and products run in OpenBLAS, whose
# kernels (chosen per CPU model) and thread partitioning change the last
# bits; drawing in a child process with the kernel type and thread count
# fixed gives the same bits on any x86-64 host with AVX2/FMA, so an input can
# be identified by its SHA-256 across machines.
# ---------------------------------------------------------------------------
PINNED_ENV = {"OPENBLAS_CORETYPE": "Haswell", "OPENBLAS_NUM_THREADS": "8", "OMP_NUM_THREADS": "8"}


def input_sha256(H: np.ndarray, S: np.ndarray) -> str:
    import hashlib

    return hashlib.sha256(np.asfortranarray(H).tobytes(order="F") + np.asfortranarray(S).tobytes(order="F")).hexdigest()


def pinned_problem(kind: str, n: int, cplx: bool, sigma_min: float, seed: int, frac: float,
                   cache_dir: str | None = None) -> tuple:
    """(Problem, sha256) of ``pencil`` (kind "pencil") or ``commuting_pencil``
    (kind "commuting") drawn in a child process with PINNED_ENV; cached as
    .npz under cache_dir (default: the system temp directory)."""
    import os
    import subprocess
    import sys
    import tempfile

    cache_dir = cache_dir or tempfile.gettempdir()
    os.makedirs(cache_dir, exist_ok=True)
    tag = "gevd_pinned_%s_%d_%s_%g_%d_%g.npz" % (kind, n, "z" if cplx else "d", sigma_min, seed, frac)
    path = os.path.join(cache_dir, tag)
    if not os.path.exists(path):
        env = dict(os.environ)
        env.update(PINNED_ENV)
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        code = ("import sys; sys.path.insert(0, %r)\n"
                "import numpy as np\n"
                "from paper_2502_02460_amd import synth\n"
                "f = synth.pencil if %r == 'pencil' else synth.commuting_pencil\n"
                "p = f(%d, %r, %r, %d, %r)\n"
                "np.savez(%r, H=p.H, S=p.S, lam=p.lam, sigma=p.sigma, k=p.k,"
                " exact=p.exact if p.exact is not None else np.zeros(0))\n") % (
                    root, kind, n, cplx, sigma_min, seed, frac, path + ".tmp.npz")
        subprocess.run([sys.executable, "-c", code], env=env, check=True)
        os.replace(path + ".tmp.npz", path)
    with np.load(path) as z:
        exact = z["exact"] if z["exact"].size else None
        p = Problem(H=np.asfortranarray(z["H"]), S=np.asfortranarray(z["S"]), k=int(z["k"]), lam=z["lam"],
                    sigma=z["sigma"], exact=exact)
    return p, input_sha256(p.H, p.S)
