"""SCF residency on the GPU: factor S once, solve with several H.

A resident solve runs exactly the kernels of the full solve after the
inversion, so its results must equal a full solve of the same (H, S)
bit for bit; they are also checked against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests import cases, floors
from tests.gpu_util import dev, host, log
from tests.linalg_checks import backward_errors, s_orthonormality

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", cases.RESIDENT)
def test_resident_equals_full_solve(gpu_lib, n, cplx):
    p, its = cases.resident_inputs(n, cplx)
    res = gpu_lib.Solver()
    full = gpu_lib.Solver()
    S_dev = dev(p.S)
    res.set_overlap(S_dev)
    assert np.array_equal(host(S_dev), p.S)  # S is not modified
    for it, (Ht, key) in enumerate(its):
        w1, C1 = res.solve_resident(dev(Ht), p.k)
        w2, C2 = full.solve(dev(Ht), dev(p.S), p.k)
        w1, C1, w2, C2 = host(w1), host(C1), host(w2), host(C2)
        assert np.array_equal(w1, w2) and np.array_equal(C1, C2)
        w_ref, _, _ = oracle.gevd(Ht, p.S, p.k)
        floors.check_eigs(w1, w_ref, p.k, floors.stored(key), f"resident n={n} cplx={cplx} it={it}:")
        eta = backward_errors(Ht, p.S, w1[: p.k], C1).max()
        log(f"  eta {eta:.2e} orth {s_orthonormality(p.S, C1):.2e}")
        assert eta < 1e-11
    res.close()
    full.close()


def test_resident_without_overlap_is_a_state_error(gpu_lib):
    s = gpu_lib.Solver()
    H = dev(np.eye(8))
    with pytest.raises(gpu_lib.GevdError) as ei:
        s.solve_resident(H, 2)
    assert ei.value.code == gpu_lib.E_STATE
    s.close()
