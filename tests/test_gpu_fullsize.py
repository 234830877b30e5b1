"""The benchmark's workloads at their full sizes (real n = 4096 and 8192 with
the lowest 30 %, complex n = 16384 with the lowest 25 %, kappa(S) ~ 1e6), in
the launch configuration bench.py times (default handle: automatic band,
persistent panels).  The CPU oracle does not finish at these sizes, so the
checks are properties that hold at any size:

* a commuting pencil (H and S built on the same Haar eigenvectors) has the
  generalized eigenvalues lam_i / sigma_i exactly, so all n computed
  eigenvalues are compared with them normwise: at complex n = 16384 (drawn
  on the device) against 1e-11 of max |eps|; at real n = 4096 and 8192
  (drawn on the CPU with pinned BLAS kernels) against max(1e-11, 2x) the
  oracle's own error on the same input (tests/golden/fullsize_oracle.json),
  with the backward error over all wanted columns held the same way;
* for the paper-shaped pencil (independent eigenvectors) and the commuting
  one, sampled eigenpairs are checked by their definitions: backward error
  ||H c - w S c|| / ((||H|| + |w| ||S||) ||c||) <= 1e-11 with the 2-norms
  known from the drawn spectra, and S-orthonormality of the sampled columns
  (<= 1e-10).

The real n = 4096 configuration is the exception: the oracle's eigenvalues
(without eigenvectors) take seconds there, so it is compared with them
eigenvalue by eigenvalue.

The sampled products run in torch (FP64 library products), not in the
solver."""
from __future__ import annotations

import json
import os

import pytest
import torch

from paper_2502_02460_amd import synth
from tests import cases, floors
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

# name, n, complex, wanted fraction, sigma_min, seed
CASES = [("real n=4096, lowest 30%", 4096, False, 0.30, 1e-6, 31),
         ("real n=8192, lowest 30%", 8192, False, 0.30, 1e-6, 33),
         ("complex n=16384, lowest 25%", 16384, True, 0.25, 1e-6, 32)]


def _sampled(H, S, w, C, k, nh, ns, count=8):
    idx = sorted(set(int(round(i * (k - 1) / (count - 1))) for i in range(count)))
    Cs = C[:, idx].contiguous()
    ws = w[idx]
    SC = S @ Cs
    R = H @ Cs - SC * ws.to(C.dtype)[None, :]
    eta = torch.linalg.vector_norm(R, dim=0) / ((nh + ws.abs() * ns) * torch.linalg.vector_norm(Cs, dim=0))
    G = Cs.conj().T @ SC
    orth = (G - torch.eye(len(idx), dtype=G.dtype, device=G.device)).abs().max()
    return float(eta.max()), float(orth)


def _solve(gpu_lib, H0, S0, k):
    s = gpu_lib.Solver()
    w, C = s.solve(H0.clone(), S0.clone(), k)
    torch.cuda.synchronize()
    s.close()
    return w, C


def test_fullsize_commuting_exact_spectrum_complex(gpu_lib):
    """complex n = 16384 (drawn on the device): all n eigenvalues against the
    exact spectrum (normwise <= 1e-11), sampled backward errors <= 1e-11."""
    name, n, cplx, frac, smin, seed = CASES[2]
    dev = torch.device("cuda:0")
    H0, S0, k, exact, lam, sigma = synth.pencil_torch(n, cplx, smin, seed, frac, dev, commuting=True,
                                                      spectra=True)
    w, C = _solve(gpu_lib, H0, S0, k)
    err = float((w - exact).abs().max() / exact.abs().max())
    eta, orth = _sampled(H0, S0, w, C, k, float(lam.abs().max()), float(sigma.max()))
    rel = float(((w[:k] - exact[:k]).abs() / exact[:k].abs()).max())
    log(f"full size, commuting pencil, {name}: all {n} eigenvalues vs exact {err:.2e} (normwise), "
        f"wanted {rel:.2e} (max relative); sampled eta {eta:.2e}, S-orthonormality {orth:.2e}")
    assert err < 1e-11
    assert eta < 1e-11
    assert orth < 1e-10


def _golden_fullsize():
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_oracle.json")) as f:
        return json.load(f)["cases"]


def _normwise_gate(g):
    """max(1e-11, 10 x the input's normwise FP64 floor): the A-1 reading
    applied to the normwise error against the exact spectrum (the oracle's
    own error on the same input is printed beside it)."""
    return max(1e-11, 10.0 * g["F_normwise"])


@pytest.mark.parametrize("n,seed", [(4096, 31), (8192, 33)])
def test_fullsize_commuting_real_against_oracle(gpu_lib, n, seed):
    """real n = 4096 and 8192 commuting pencils drawn on the CPU with pinned
    BLAS kernels (tests/golden/make_fullsize.py ran the oracle on the same
    draw, SHA-256 recorded): the GPU's normwise eigenvalue error against the
    exact spectrum within max(1e-11, 10 x the input's normwise floor F_n),
    its largest backward error over all k wanted columns within
    max(1e-11, 2x) the oracle's own on that input, sampled S-orthonormality
    within max(1e-10, 10x) the oracle's.  At kappa(S) = 1e6
    the backward error of the Cholesky route is limited by the standard
    solver's residual relative to ||A|| ~ 5e7, which puts the oracle's own
    value near 1e-11."""
    p, sha = synth.pinned_problem("commuting", n, False, 1e-6, seed, 0.3)
    g = _golden_fullsize()["commuting/n=%d/d/smin=1e-06/seed=%d/f=0.3" % (n, seed)]
    assert "F_normwise" in g, "run python tests/golden/make_fullsize.py --floors"
    same = sha == g["sha256"]
    k = p.k
    dev = torch.device("cuda:0")
    H0 = torch.from_numpy(p.H).to(dev)
    S0 = torch.from_numpy(p.S).to(dev)
    w, C = _solve(gpu_lib, H0, S0, k)
    exact = torch.from_numpy(p.exact).to(dev)
    err = float((w - exact).abs().max() / exact.abs().max())
    nh, ns = float(abs(p.lam).max()), float(p.sigma.max())
    R = H0 @ C - (S0 @ C) * w[:k][None, :]
    eta_all = R.norm(dim=0) / ((nh + w[:k].abs() * ns) * C.norm(dim=0))
    eta_max = float(eta_all.max())
    idx = g["sample_index"]
    Cs = C[:, idx].contiguous()
    orth = float((Cs.mT @ (S0 @ Cs) - torch.eye(len(idx), dtype=Cs.dtype, device=dev)).abs().max())
    log(f"full size, commuting pencil, real n={n}: input {'identical to' if same else 'NOT bit-identical to'} "
        f"the oracle's draw; eigenvalues vs exact {err:.2e} normwise (oracle {g['eig_err_normwise']:.2e}, "
        f"floor {g['F_normwise']:.2e}); "
        f"max eta over all {k} wanted {eta_max:.2e} (oracle {g['eta_max_all']:.2e}); "
        f"sampled S-orthonormality {orth:.2e} (oracle {g['orth_sampled']:.2e})")
    assert err <= _normwise_gate(g)
    assert eta_max <= max(1e-11, 2.0 * g["eta_max_all"])
    assert orth <= max(1e-10, 10.0 * g["orth_sampled"])


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fullsize_paper_pencil_sampled(gpu_lib, case):
    name, n, cplx, frac, smin, seed = case
    dev = torch.device("cuda:0")
    H0, S0, k, _, lam, sigma = synth.pencil_torch(n, cplx, smin, seed + 100, frac, dev, spectra=True)
    w, C = _solve(gpu_lib, H0, S0, k)
    assert bool((w[1:] >= w[:-1]).all())  # ascending
    eta, orth = _sampled(H0, S0, w, C, k, float(lam.abs().max()), float(sigma.max()))
    log(f"full size, paper-shaped pencil, {name}: sampled eta {eta:.2e}, S-orthonormality {orth:.2e}")
    assert eta < 1e-11
    assert orth < 1e-10


def test_fullsize_c1_oracle_parity(gpu_lib):
    """The real n = 4096 benchmark configuration (lowest 30 %, kappa(S) ~
    1e6), drawn on the CPU, solved in the launch configuration bench.py times
    (b = 64, persistent panels, eight-wave tiles where the shapes allow), and
    compared with the oracle's eigenvalues of the same input (its route
    without eigenvectors): each wanted eigenvalue within max(1e-12, 10 F) of
    the oracle's, all n within 1e-11 normwise; sampled backward errors and
    S-orthonormality of the eigenvectors."""
    p, key = cases.config_pencil("c1")
    n, k = p.H.shape[0], p.k
    w_ref = floors.oracle_eigenvalues(p.H, p.S)
    dev = torch.device("cuda:0")
    H0 = torch.from_numpy(p.H).to(dev)
    S0 = torch.from_numpy(p.S).to(dev)
    assert H0.stride(0) == 1 and S0.stride(0) == 1  # column-major, as drawn
    w, C = _solve(gpu_lib, H0, S0, k)
    floors.check_eigs(w.cpu().numpy(), w_ref, k, floors.stored(key), f"full size c1 n={n} k={k}:")
    eta, orth = _sampled(H0, S0, w, C, k, float(abs(p.lam).max()), float(p.sigma.max()), count=16)
    log(f"  sampled eta {eta:.2e}, S-orthonormality {orth:.2e}")
    assert eta < 1e-11
    assert orth < 1e-10


def test_fullsize_precision_form_error_stated(gpu_lib):
    """The reduced-precision form (FP32 products in full -> band and the
    stage-1 back-transformation, FP64 refinement of the wanted pairs) at the
    real n = 8192 shape, on the pinned commuting pencil of
    test_fullsize_commuting_real_against_oracle: its eigenvalue error against
    the exact spectrum is stated and bounded by what the method delivers (the
    FP32 stages limit it; the FP64 target is not reached, see the precision
    tests); the FP64 form on the same input is held to the FP64 gate."""
    n, seed = 8192, 33
    p, _ = synth.pinned_problem("commuting", n, False, 1e-6, seed, 0.3)
    g = _golden_fullsize()["commuting/n=%d/d/smin=1e-06/seed=%d/f=0.3" % (n, seed)]
    k = p.k
    dev = torch.device("cuda:0")
    H0 = torch.from_numpy(p.H).to(dev)
    S0 = torch.from_numpy(p.S).to(dev)
    exact = torch.from_numpy(p.exact).to(dev)
    s = gpu_lib.Solver(precision="fp32+refine")
    w, C = s.solve(H0.clone(), S0.clone(), k)
    torch.cuda.synchronize()
    s.close()
    w64, _ = _solve(gpu_lib, H0, S0, k)
    scale = exact.abs().max()
    err = float((w[:k] - exact[:k]).abs().max() / scale)
    err64 = float((w64[:k] - exact[:k]).abs().max() / scale)
    eta, orth = _sampled(H0, S0, w, C, k, float(abs(p.lam).max()), float(p.sigma.max()))
    log(f"full size, precision form, real n={n}: wanted eigenvalues vs exact {err:.2e} normwise "
        f"(FP64 form {err64:.2e}); sampled eta {eta:.2e}, S-orthonormality {orth:.2e}")
    assert err64 <= _normwise_gate(g)
    assert err < 1e-6
