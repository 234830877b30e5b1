"""Serving scheduler on the CPU with a simulated device: service time
proportional to the solve's flops, so admission, batching and latency
accounting are checked deterministically without a GPU."""
from __future__ import annotations

import threading
import time

import numpy as np

from paper_2502_02460_amd import serve


def fake_device(scale=2e-12):
    lock = threading.Lock()
    live = {"bytes": 0, "max": 0}

    def service(r):
        es = 4.0 if r.cplx else 1.0
        return scale * es * (8 * r.n ** 3 / 3 + 5 * r.n ** 2 * r.k)

    def run_request(r, on_solve, t0):
        submit = r.arrival
        for it in range(r.iters):
            time.sleep(service(r))
            done = time.perf_counter() - t0
            on_solve(serve.SolveRecord(r.rid, it, r.n, r.cplx, submit, done))
            submit = done

    def run_batch(rs, on_solve, t0):
        submits = [r.arrival for r in rs]
        for it in range(max(r.iters for r in rs)):
            time.sleep(max(service(r) for r in rs))
            done = time.perf_counter() - t0
            for i, r in enumerate(rs):
                if it < r.iters:
                    on_solve(serve.SolveRecord(r.rid, it, r.n, r.cplx, submits[i], done, batched=True))
                    submits[i] = done

    return run_request, run_batch


def test_poisson_stream_shape():
    reqs = serve.poisson_stream(2000, 200.0, seed=4)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / 200.0) < 0.1 / 200.0
    small = np.array([r.n <= 512 for r in reqs])
    assert 0.65 < small.mean() < 0.75
    assert 0.55 < np.mean([r.cplx for r in reqs]) < 0.65
    assert all(64 <= r.n <= 8192 for r in reqs)
    assert all(r.k == int(np.ceil(0.3 * r.n - 1e-9)) for r in reqs)


def test_scheduler_serves_everything_within_budget():
    reqs = serve.poisson_stream(60, 400.0, seed=7, large=(600, 1200), iters=3)
    run_request, run_batch = fake_device()
    ws = lambda r: 1000 * r.n
    budget = 3 * max(serve.footprint_bytes(r, ws(r)) for r in reqs)
    sched = serve.Scheduler(budget, large_workers=3, small_workers=2, small_n=512, workspace_of=ws,
                            executor=run_request, batch_executor=run_batch, batch=4, batch_wait=0.01)
    res = sched.run(reqs)
    assert len(res.records) == sum(r.iters for r in reqs)
    assert res.peak_bytes <= budget
    # every request's iterations are consecutive and causal
    by = {}
    for rec in res.records:
        by.setdefault(rec.rid, []).append(rec)
    for r in reqs:
        recs = sorted(by[r.rid], key=lambda x: x.it)
        assert [x.it for x in recs] == list(range(r.iters))
        assert recs[0].submit == r.arrival
        for a, b in zip(recs, recs[1:]):
            assert b.submit == a.done and b.done >= b.submit
    s = res.summary()
    assert s["solves"] == len(res.records) and s["p99_s"] >= s["p50_s"] > 0
    # small requests were batched
    assert any(rec.batched for rec in res.records)


def test_admission_defers_when_memory_is_short():
    reqs = [serve.Request(i, False, 1000, 300, 0.001 * i, seed=i, iters=1) for i in range(6)]
    run_request, run_batch = fake_device(scale=5e-11)
    ws = lambda r: 0
    one = serve.footprint_bytes(reqs[0], 0)
    sched = serve.Scheduler(2 * one, large_workers=6, small_workers=1, small_n=512, workspace_of=ws,
                            executor=run_request, batch_executor=run_batch)
    res = sched.run(reqs)
    assert res.peak_bytes <= 2 * one
    assert res.deferred >= 1
    assert len(res.records) == 6
    # first come first served
    first = sorted(res.records, key=lambda x: x.done)
    starts = sorted(reqs, key=lambda r: r.arrival)
    assert first[0].rid in (starts[0].rid, starts[1].rid)


def test_worker_failures_are_reported():
    reqs = serve.poisson_stream(12, 400.0, seed=9, large=(600, 900), iters=2)
    run_request, run_batch = fake_device()

    def failing(r, on_solve, t0):
        if r.rid % 3 == 0:
            raise RuntimeError("device error for %d" % r.rid)
        run_request(r, on_solve, t0)

    sched = serve.Scheduler(1 << 40, large_workers=2, small_workers=1, small_n=512, workspace_of=lambda r: 0,
                            executor=failing, batch_executor=run_batch, batch=4, batch_wait=0.01)
    res = sched.run(reqs)
    bad = sorted(rid for rids, _ in res.errors for rid in rids)
    assert bad == sorted(r.rid for r in reqs if r.n > 512 and r.rid % 3 == 0)
    assert res.summary()["errors"] == len(bad)
    ok = [r for r in reqs if r.rid not in bad]
    assert len(res.records) == sum(r.iters for r in ok)


def test_progress_reports_every_finished_request():
    reqs = serve.poisson_stream(20, 400.0, seed=9, large=(600, 900), iters=2)
    run_request, run_batch = fake_device()
    seen = []
    lock = threading.Lock()

    def progress(done, total, secs):
        with lock:
            seen.append((done, total, secs))

    sched = serve.Scheduler(1 << 40, large_workers=2, small_workers=1, small_n=512, workspace_of=lambda r: 0,
                            executor=run_request, batch_executor=run_batch, batch=4, batch_wait=0.01,
                            progress=progress)
    res = sched.run(reqs)
    assert len(res.records) == sum(r.iters for r in reqs)
    assert seen and all(t == len(reqs) for _, t, _ in seen)
    counts = sorted(d for d, _, _ in seen)
    assert counts[-1] == len(reqs)  # the last report covers every request
    assert all(b > a for a, b in zip(counts, counts[1:]))  # one report per finished launch
    assert all(s >= 0.0 for _, _, s in seen)
