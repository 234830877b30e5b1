"""Batched small problems (n <= 512) in the fused persistent kernel.

Parity against the oracle problem by problem (each wanted eigenvalue within
max(1e-12, 10 F) of the oracle's, F the input's FP64 floor, all within 1e-11
normwise; backward error, S-orthonormality; the gates of the single solve);
every result of a mixed batch equals the same problem solved alone, bit for
bit (each problem is one workgroup's work, independent of its neighbours);
graph replays equal the eager launch; a failing problem reports its own
status and leaves the rest intact; the shape tuner returns a valid shape."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2502_02460_amd import synth
from tests import cases, floors
from tests.gpu_util import dev, host, log
from tests.linalg_checks import backward_errors, s_orthonormality

pytestmark = pytest.mark.gpu

# (n, complex, sigma_min, fraction wanted): bucket edges, ragged orders,
# the degenerate n = 1 and 2, and the largest order
MIX = [(1, False, 1e-3, 1.0), (2, True, 1e-3, 1.0), (7, False, 1e-3, 1.0), (64, True, 1e-6, 0.3),
       (65, False, 1e-6, 0.3), (128, False, 1e-3, 1.0), (130, True, 1e-6, 0.3), (256, True, 1e-6, 0.3),
       (257, False, 1e-6, 0.3), (512, False, 1e-6, 0.3), (512, True, 1e-6, 0.3), (333, True, 1e-3, 0.5)]


def _pencils():
    return [synth.pencil(n, c, smin, 4000 + i, frac) for i, (n, c, smin, frac) in enumerate(MIX)]


def _items(ps):
    return [(dev(p.H), dev(p.S), p.k) for p in ps]


@pytest.fixture(scope="module")
def solver(gpu_lib):
    s = gpu_lib.Solver()
    yield s
    s.close()


def test_batched_matches_oracle(solver):
    pk = cases.batched_pencils()
    ps = [p for p, _ in pk]
    res, info = solver.solve_batched(_items(ps))
    assert info == [0] * len(ps)
    for (p, key), (w, C) in zip(pk, res):
        w, C = host(w), host(C)
        w_ref, C_ref, _ = oracle.gevd(p.H, p.S, p.k)
        floors.check_eigs(w, w_ref, p.k, floors.stored(key),
                          f"batched n={p.H.shape[0]} k={p.k} cplx={np.iscomplexobj(p.H)}:")
        eta = backward_errors(p.H, p.S, w[: p.k], C).max()
        orth, orth_ref = s_orthonormality(p.S, C), s_orthonormality(p.S, C_ref)
        log(f"  eta {eta:.2e} orth {orth:.2e} (oracle {orth_ref:.2e})")
        assert eta < 1e-11
        assert orth < max(1e-11, 10 * orth_ref)


def test_batched_equals_alone_and_graph_replay(solver):
    ps = _pencils()
    res, info = solver.solve_batched(_items(ps))
    assert info == [0] * len(ps)
    mix = [(host(w), host(C)) for w, C in res]
    for i in (0, 3, 9, 10):  # alone, one at a time
        (w, C), = solver.solve_batched([_items([ps[i]])[0]])[0]
        assert np.array_equal(host(w), mix[i][0]) and np.array_equal(host(C), mix[i][1])
    # captured batch over fixed buffers, inputs rewritten before each replay
    items = _items(ps)
    pristine = [(H.clone(), S.clone()) for H, S, _ in items]
    b = solver.batch(items)
    for rep in range(3):
        for (H, S, _), (H0, S0) in zip(items, pristine):
            H.copy_(H0)
            S.copy_(S0)
        torch.cuda.synchronize()
        assert b.run() == [0] * len(ps)
        for (w, C), (w0, C0) in zip(b.results, mix):
            assert np.array_equal(host(w), w0) and np.array_equal(host(C), C0)
        log(f"graph replay {rep}: identical to the eager batch")
    b.close()


def test_failures_stay_local(solver):
    ps = [synth.pencil(n, c, 1e-3, 77 + n, 0.5) for n, c in ((40, False), (90, True), (200, False))]
    items = _items(ps)
    bad_S = ps[1].S.copy()
    bad_S[5, 5] = -1.0  # leading minor 6 is not positive definite
    items[1] = (dev(ps[1].H), dev(bad_S), ps[1].k)
    bad_H = ps[2].H.copy()
    bad_H[3, 10] = np.nan
    items[2] = (dev(bad_H), dev(ps[2].S), ps[2].k)
    items.append(_items([ps[0]])[0])
    res, info = solver.solve_batched(items)
    assert info[0] == 0 and info[3] == 0
    assert info[1] > 0 and info[1] <= 6
    assert info[2] == -1001
    assert np.array_equal(host(res[0][0]), host(res[3][0]))


def test_async_replay_status_on_device(solver):
    """gevd_batch_run_async: no host synchronisation; the statuses land in a
    device array on the stream (a failing problem included), the results
    equal those of the synchronous replay bit for bit."""
    ps = [synth.pencil(n, c, 1e-3, 91 + n, 0.5) for n, c in ((48, True), (100, False), (160, True))]
    items = _items(ps)
    bad_S = ps[1].S.copy()
    bad_S[7, 7] = -1.0  # leading minor 8 is not positive definite
    items[1] = (items[1][0], dev(bad_S), ps[1].k)
    pristine = [(H.clone(), S.clone()) for H, S, _ in items]
    b = solver.batch(items)
    info_sync = b.run()
    assert info_sync[0] == 0 and info_sync[2] == 0 and 0 < info_sync[1] <= 8
    ref = [(host(w), host(C)) for w, C in b.results]
    info_dev = torch.full((len(items),), -77, dtype=torch.int32, device="cuda")
    for rep in range(2):
        for (H, S, _), (H0, S0) in zip(items, pristine):
            H.copy_(H0)
            S.copy_(S0)
        info_dev.fill_(-77)
        b.run_async(info_dev)
        got = info_dev.cpu().tolist()  # stream-ordered after the replay
        assert got == info_sync, (rep, got, info_sync)
        for i in (0, 2):
            assert np.array_equal(host(b.results[i][0]), ref[i][0])
            assert np.array_equal(host(b.results[i][1]), ref[i][1])
    with pytest.raises(ValueError):
        b.run_async(torch.zeros(len(items) - 1, dtype=torch.int32, device="cuda"))
    b.close()


def test_degenerate_spectrum(solver):
    """Eigenvalues of multiplicity two and three (S = I, H = Q diag(lam) Q^H
    with Haar Q): the twisted-factorisation vectors of a repeated eigenvalue
    coincide, so the problem must come out of the QL fallback (or of the
    cluster orthogonalisation) with exact eigenvalues, small backward errors
    and orthonormal vectors, like any other."""
    rng = np.random.default_rng(4242)
    items, ref = [], []
    for n, cplx, mult in ((48, False, 2), (60, True, 3), (96, True, 2)):
        lam = np.repeat(np.arange(1.0, n // mult + 1.0), mult)
        q = synth.haar(n, rng, cplx)
        H = np.asfortranarray((q * lam) @ q.conj().T)
        H = 0.5 * (H + H.conj().T)
        S = np.asfortranarray(np.eye(n, dtype=H.dtype))
        k = n // 2
        items.append((dev(H), dev(S), k))
        ref.append((H, S, np.sort(lam), k))
    res, info = solver.solve_batched(items)
    assert info == [0] * len(items)
    for (H, S, lam, k), (w, C) in zip(ref, res):
        w, C = host(w), host(C)
        err = np.abs(w - lam).max() / np.abs(lam).max()
        eta = backward_errors(H, S, w[:k], C).max()
        orth = s_orthonormality(S, C)
        log(f"  degenerate n={H.shape[0]}: eig err {err:.1e} eta {eta:.1e} orth {orth:.1e}")
        assert err < 1e-13
        assert eta < 1e-12
        assert orth < 1e-12


def test_tuner_and_shapes(gpu_lib, solver):
    t, w = solver.tune_batched(torch.float64, 60, count=96)
    assert t in (64, 128, 256, 512, 1024) and w >= 1
    assert solver.batch_shape(torch.float64, 33) == (t, w)
    p = synth.pencil(60, False, 1e-3, 5, 1.0)
    (wv, C), = solver.solve_batched(_items([p]))[0]
    w_ref, _, _ = oracle.gevd(p.H, p.S, p.k)
    floors.check_eigs(host(wv), w_ref, p.k, floors.floor(p.H, p.S, p.k), "tuned shape n=60:")
    solver.set_batch_shape(torch.float64, 60, 0, 0)  # back to the default
    log(f"tuned shape for real n<=64: {t} lanes, {w} workgroups per CU")


def test_result_independent_of_launch_shape(solver):
    """Reductions inside the fused kernel run in a fixed order, so the launch
    shape (lanes per workgroup, workgroups per CU) changes speed only."""
    ps = [synth.pencil(n, c, 1e-6, 300 + n, 0.3) for n, c in ((100, False), (300, True), (480, False))]
    outs = []
    for threads, wg in ((64, 4), (256, 1), (512, 1), (1024, 1)):
        for dt in (torch.float64, torch.complex128):
            for n in (64, 128, 256, 512):
                solver.set_batch_shape(dt, n, threads, wg)
        res, info = solver.solve_batched(_items(ps))
        assert info == [0] * len(ps)
        outs.append([(host(w), host(C)) for w, C in res])
    for dt in (torch.float64, torch.complex128):
        for n in (64, 128, 256, 512):
            solver.set_batch_shape(dt, n, 0, 0)
    for other in outs[1:]:
        for (w0, C0), (w1, C1) in zip(outs[0], other):
            assert np.array_equal(w0, w1) and np.array_equal(C0, C1)
