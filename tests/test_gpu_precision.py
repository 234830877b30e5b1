"""The reduced-precision form: FP32 matrix-core products in the full -> band
reduction and the stage-1 back-transformation, then FP64 refinement of the
wanted pairs (Ogita-Aishima correction restricted to their subspace).

The target of this form is the FP64 accuracy: each wanted eigenvalue
within max(1e-12, 10 F) of the oracle's (F the input's FP64 floor) and
backward errors <= 1e-11.  test_precision_form_meets_fp64_targets asserts
exactly that and is marked xfail(strict=True) while the refinement does not
reach it (measured: see its reason); it turns into a failure the moment it
passes, so the mark cannot outlive the fix.

The other tests assert what the current form delivers: (1) the FP32 stages
alone give FP32-level results; (2) when the wanted subspace is well
separated from the rest of the spectrum, refinement brings the eigenvalues
to the 1e-11 (normwise) level, while the eigenvector residual and
S-orthonormality stay at the level of the FP32 stages; (3) for the
paper-shaped pencils (kappa(S) = 1e6) the results are reported against the
oracle, and refinement must not make them worse."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2502_02460_amd import synth
from tests import floors
from tests.gpu_util import dev, host, log
from tests.linalg_checks import backward_errors, s_orthonormality

pytestmark = pytest.mark.gpu


def _gapped_pencil(n, cplx, k, seed):
    """H c = eps S c with the wanted k eigenvalues in [-10, -5] and the rest
    in [5, 10] (a relative gap of about 1 at the subspace boundary), S with
    kappa = 100."""
    rng = np.random.default_rng(seed)
    V = synth.haar(n, rng, cplx)
    W = synth.haar(n, rng, cplx)
    sigma = np.exp(rng.uniform(np.log(1e-2), 0.0, n))
    S = (V * sigma) @ V.conj().T
    eps = np.concatenate([rng.uniform(-10, -5, k), rng.uniform(5, 10, n - k)])
    # H = S^{1/2} W diag(eps) W^H S^{1/2} has generalized eigenvalues eps
    Sh = (V * np.sqrt(sigma)) @ V.conj().T
    H = Sh @ ((W * eps) @ W.conj().T) @ Sh
    H = 0.5 * (H + H.conj().T)
    S = 0.5 * (S + S.conj().T)
    return H, S, np.sort(eps)


def _run(gpu_lib, H, S, k, precision, refine=2):
    s = gpu_lib.Solver(precision=precision, refine=refine)
    w, C = s.solve(dev(H), dev(S), k)
    s.close()
    return host(w), host(C)


@pytest.mark.parametrize("cplx", [False, True])
def test_refinement_on_separated_subspace(gpu_lib, cplx):
    n, k = 768, 200
    H, S, eps = _gapped_pencil(n, cplx, k, 11 + cplx)
    w0, C0 = _run(gpu_lib, H, S, k, "fp32+refine", refine=0)
    w2, C2 = _run(gpu_lib, H, S, k, "fp32+refine", refine=2)
    wd, Cd = _run(gpu_lib, H, S, k, "fp64")
    nrm = np.abs(eps).max()
    e0 = np.abs(w0[:k] - eps[:k]).max() / nrm
    e2 = np.abs(w2[:k] - eps[:k]).max() / nrm
    ed = np.abs(wd[:k] - eps[:k]).max() / nrm
    h0 = backward_errors(H, S, w0[:k], C0).max()
    h2 = backward_errors(H, S, w2[:k], C2).max()
    o2 = s_orthonormality(S, C2)
    log(f"gapped n={n} k={k} cplx={cplx}: eig fp32 {e0:.2e} refined {e2:.2e} fp64 {ed:.2e}; "
        f"eta fp32 {h0:.2e} refined {h2:.2e}; orth refined {o2:.2e}")
    assert e0 < 1e-5
    assert e2 < 1e-11 and e2 <= e0
    assert h2 <= 1.1 * h0 and h2 < 1e-5
    assert o2 < 1e-4


@pytest.mark.parametrize("n,cplx,smin", [(1024, False, 1e-6), (512, True, 1e-6), (1024, False, 1e-2)])
def test_paper_shaped_pencil_reported(gpu_lib, n, cplx, smin):
    p = synth.pencil(n, cplx, smin, 70 + n, 0.3)
    w_ref, C_ref, _ = oracle.gevd(p.H, p.S, p.k)
    nrm = np.abs(w_ref).max()
    out = {}
    for prec, rf in (("fp64", 0), ("fp32+refine", 0), ("fp32+refine", 2)):
        w, C = _run(gpu_lib, p.H, p.S, p.k, prec, rf)
        out[(prec, rf)] = (np.abs(w[: p.k] - w_ref[: p.k]).max() / nrm,
                           backward_errors(p.H, p.S, w[: p.k], C).max())
    (ed, hd), (e0, h0), (e2, h2) = out[("fp64", 0)], out[("fp32+refine", 0)], out[("fp32+refine", 2)]
    log(f"paper-shaped n={n} cplx={cplx} sigma_min={smin}: eig fp64 {ed:.2e} fp32 {e0:.2e} refined {e2:.2e}; "
        f"eta fp64 {hd:.2e} fp32 {h0:.2e} refined {h2:.2e}")
    assert ed < 1e-11
    assert e0 < 1e-6            # FP32 stages: normwise error at FP32 level
    assert e2 <= 2.0 * e0       # refinement does not make it materially worse
    assert h2 <= 1.1 * h0


@pytest.mark.xfail(strict=True, reason="the subspace refinement cannot restore components the FP32 stages lost "
                                       "outside span(X): measured relative eigenvalue error ~1e-6..1e-4 and eta "
                                       "~1e-7..3e-4 at kappa(S) = 1e6 against the FP64 targets")
@pytest.mark.parametrize("n,cplx", [(1024, False), (512, True)])
def test_precision_form_meets_fp64_targets(gpu_lib, n, cplx):
    p = synth.pencil(n, cplx, 1e-6, 70 + n, 0.3)
    w_ref, _, _ = oracle.gevd(p.H, p.S, p.k)
    w, C = _run(gpu_lib, p.H, p.S, p.k, "fp32+refine", 2)
    eta = backward_errors(p.H, p.S, w[: p.k], C).max()
    log(f"precision form n={n} cplx={cplx}: eta {eta:.2e}")
    floors.check_eigs(w, w_ref, p.k, floors.floor(p.H, p.S, p.k), f"precision form n={n} cplx={cplx}:")
    assert eta < 1e-11
