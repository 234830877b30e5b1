"""Serving loop for streams of generalized eigensolves (k-points, spin
channels), with SCF residency and admission by device-memory footprint.

The paper's ELSI layer treats independent k-point and spin problems as
trivially parallel work (Figure 1 caption, section "ELPA - Usability").  Here
such problems arrive over time on one GPU and are served concurrently:

* each request carries an (H, S) pair of order n (real or complex) and wants
  its lowest k eigenpairs for several SCF iterations; S stays fixed, so its
  factor U^{-1} is computed once per request and kept on the device
  (gevd_set_overlap), and every iteration is a resident solve with the
  iteration's H (gevd_solve_resident);
* a request is admitted when a worker of its size class is free and its
  device-memory footprint (inputs, outputs, the handle's workspace and the
  resident factor) fits the budget; otherwise it waits, first come first
  served within its class, and is admitted as soon as memory frees up;
* workers are host threads, each owning a library handle on its own HIP
  stream, so admitted requests' kernels overlap on the device while the
  scheduler keeps accepting arrivals;
* small requests (n <= small_n) are served together: up to `batch` of them
  are collected into one batch (launched when full or when the oldest has
  waited `batch_wait` seconds) and run by the batched entry point.

Latency of a solve is measured from its arrival (the request's arrival for
the first SCF iteration, the previous iteration's result for the others) to
its result.  The scheduler itself is plain Python and is tested on the CPU
with a simulated device (see tests/test_serve.py).
"""
from __future__ import annotations

import heapq
import math
import queue
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    cplx: bool
    n: int
    k: int
    arrival: float  # seconds from the start of the stream
    seed: int
    iters: int = 5
    sigma_min: float = 1e-6


@dataclass
class SolveRecord:
    rid: int
    it: int
    n: int
    cplx: bool
    submit: float
    done: float
    batched: bool = False

    @property
    def latency(self) -> float:
        return self.done - self.submit


@dataclass
class StreamResult:
    records: list = field(default_factory=list)
    makespan: float = 0.0
    deferred: int = 0  # admissions postponed for memory
    peak_bytes: int = 0
    results: dict = field(default_factory=dict)  # rid -> list of (eval, C) per iteration (if kept)
    errors: list = field(default_factory=list)   # (request ids, message) of failed work

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.records]) if self.records else np.zeros(1)
        by = {}
        for name, sel in (("small", lambda r: r.batched), ("large", lambda r: not r.batched)):
            ls = np.array([r.latency for r in self.records if sel(r)])
            if ls.size:
                by[name] = {"solves": int(ls.size), "p50_s": float(np.percentile(ls, 50)),
                            "p99_s": float(np.percentile(ls, 99))}
        return {
            "by_class": by,
            "solves": len(self.records),
            "solves_per_s": len(self.records) / self.makespan if self.makespan > 0 else 0.0,
            "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)),
            "max_s": float(lat.max()),
            "makespan_s": self.makespan,
            "deferred_admissions": self.deferred,
            "peak_admitted_bytes": self.peak_bytes,
            "errors": len(self.errors),
        }


def poisson_stream(count: int, rate: float, seed: int = 4, small=(64, 512), large=(1024, 8192),
                   frac_small: float = 0.7, frac_complex: float = 0.6, frac_wanted: float = 0.3,
                   iters: int = 5) -> list[Request]:
    """Requests with exponential inter-arrival gaps (mean 1/rate), sizes 70 %
    uniform in `small` and 30 % uniform in `large`, 60 % complex."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        lo, hi = small if rng.random() < frac_small else large
        n = int(rng.integers(lo, hi + 1))
        cplx = bool(rng.random() < frac_complex)
        k = max(1, int(math.ceil(frac_wanted * n - 1e-9)))
        out.append(Request(rid, cplx, n, k, t, seed=1_000_003 * seed + rid, iters=iters))
    return out


def footprint_bytes(req: Request, workspace: int) -> int:
    """Device bytes a request holds while admitted: H0, S, the iteration's H,
    C, the eigenvalues, the resident U^{-1}, and the handle workspace."""
    es = 16 if req.cplx else 8
    n, k = req.n, req.k
    return es * (4 * n * n + n * k) + 8 * n + workspace


class Scheduler:
    """Admission and dispatch (device-independent).

    `executor(req, on_solve)` runs one request's SCF iterations on a worker
    and calls `on_solve(record)` after each; `batch_executor(reqs, on_solve)`
    runs a batch of small requests together.  Both run on worker threads."""

    def __init__(self, budget_bytes: int, large_workers: int, small_workers: int, small_n: int,
                 workspace_of, executor, batch_executor=None, batch: int = 8, batch_wait: float = 0.02,
                 clock=time.perf_counter, progress=None):
        self.budget = budget_bytes
        self.workspace_of = workspace_of
        self.executor = executor
        self.batch_executor = batch_executor
        self.batch = batch
        self.batch_wait = batch_wait
        self.small_n = small_n
        self.clock = clock
        self.free = {"large": large_workers, "small": small_workers}
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.in_use = 0
        self.result = StreamResult()
        self.progress = progress  # called as progress(done, total, seconds) after each finished request

    def _cls(self, req: Request) -> str:
        return "small" if req.n <= self.small_n else "large"

    def run(self, requests: list[Request]) -> StreamResult:
        reqs = sorted(requests, key=lambda r: r.arrival)
        waiting = {"large": [], "small": []}  # FIFO lists
        threads = []
        t0 = self.clock()
        nxt = 0
        deferred_ids = set()
        outstanding = len(reqs)
        done_count = [0]

        def on_solve(rec: SolveRecord):
            with self.lock:
                self.result.records.append(rec)

        def finish(cost: int, cls: str, n_req: int):
            with self.cv:
                self.in_use -= cost
                self.free[cls] += 1
                done_count[0] += n_req
                done = done_count[0]
                self.cv.notify_all()
            if self.progress is not None:
                self.progress(done, outstanding, self.clock() - t0)

        def launch(cls: str, batch_reqs: list[Request]):
            cost = sum(footprint_bytes(r, self.workspace_of(r)) for r in batch_reqs)
            self.in_use += cost
            self.free[cls] -= 1
            self.result.peak_bytes = max(self.result.peak_bytes, self.in_use)

            def body():
                try:
                    if len(batch_reqs) > 1 or (cls == "small" and self.batch_executor is not None):
                        self.batch_executor(batch_reqs, on_solve, t0)
                    else:
                        self.executor(batch_reqs[0], on_solve, t0)
                except Exception as exc:  # reported in the result, not lost with the thread
                    with self.lock:
                        self.result.errors.append(([r.rid for r in batch_reqs], repr(exc)))
                finally:
                    finish(cost, cls, len(batch_reqs))

            th = threading.Thread(target=body, daemon=True)
            th.start()
            threads.append(th)

        with self.cv:
            while done_count[0] < outstanding:
                now = self.clock() - t0
                while nxt < len(reqs) and reqs[nxt].arrival <= now:
                    waiting[self._cls(reqs[nxt])].append(reqs[nxt])
                    nxt += 1
                # large: first come first served, one request per worker
                while waiting["large"] and self.free["large"] > 0:
                    r = waiting["large"][0]
                    cost = footprint_bytes(r, self.workspace_of(r))
                    if self.in_use + cost > self.budget and self.in_use > 0:
                        if r.rid not in deferred_ids:
                            deferred_ids.add(r.rid)
                            self.result.deferred += 1
                        break
                    waiting["large"].pop(0)
                    launch("large", [r])
                # small: batches, launched full or after batch_wait
                while waiting["small"] and self.free["small"] > 0:
                    oldest = waiting["small"][0].arrival
                    if len(waiting["small"]) < self.batch and now - oldest < self.batch_wait and nxt < len(reqs):
                        break
                    take = waiting["small"][: self.batch]
                    cost = sum(footprint_bytes(r, self.workspace_of(r)) for r in take)
                    if self.in_use + cost > self.budget and self.in_use > 0:
                        if take[0].rid not in deferred_ids:
                            deferred_ids.add(take[0].rid)
                            self.result.deferred += 1
                        break
                    del waiting["small"][: len(take)]
                    launch("small", take)
                # sleep until the next arrival, a completion, or a batch deadline
                timeout = 0.05
                if nxt < len(reqs):
                    timeout = min(timeout, max(0.0, reqs[nxt].arrival - now))
                if waiting["small"]:
                    timeout = min(timeout, max(0.0, waiting["small"][0].arrival + self.batch_wait - now))
                self.cv.wait(timeout=max(timeout, 1e-4))
        for th in threads:
            th.join()
        self.result.makespan = self.clock() - t0
        self.result.records.sort(key=lambda r: (r.submit, r.rid, r.it))
        return self.result


# ---------------------------------------------------------------------------
# GPU side: inputs, workers, the stream driver
# ---------------------------------------------------------------------------

def _structured_unitary_apply(M, gen, cplx: bool, nrefl: int = 8):
    """M <- Q M Q^H for Q a product of nrefl random Householder reflectors and
    a random diagonal phase (fast O(nrefl n^2) stand-in for a Haar unitary,
    used for the serving stream where drawing thousands of Haar matrices of
    order up to 8192 would dominate the run)."""
    import torch

    n = M.shape[0]
    dt = M.dtype
    for _ in range(nrefl):
        v = torch.randn(n, dtype=torch.float64, device=M.device, generator=gen)
        if cplx:
            v = v + 1j * torch.randn(n, dtype=torch.float64, device=M.device, generator=gen)
        v = (v / v.norm()).to(dt)
        # (I - 2 v v^H) M (I - 2 v v^H)
        M = M - 2.0 * torch.outer(v, v.conj() @ M)
        M = M - 2.0 * torch.outer(M @ v, v.conj())
    if cplx:
        ph = torch.exp(1j * 2 * math.pi * torch.rand(n, dtype=torch.float64, device=M.device, generator=gen))
        M = ph[:, None] * M * ph.conj()[None, :]
    return M


def request_inputs(req: Request, device):
    """(H0, S) of a request, drawn on the device: spectra as in the paper-
    shaped generator (sigma log-uniform in [sigma_min, 1]; 10 % core-like
    eigenvalues in [-50, -5], the rest in [-1, 3]) with structured unitaries."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(req.seed)
    n = req.n
    dt = torch.complex128 if req.cplx else torch.float64
    sigma = torch.exp(torch.rand(n, dtype=torch.float64, device=device, generator=gen) * math.log(req.sigma_min))
    nc = int(round(0.1 * n))
    lam = torch.cat([-50.0 + 45.0 * torch.rand(nc, dtype=torch.float64, device=device, generator=gen),
                     -1.0 + 4.0 * torch.rand(n - nc, dtype=torch.float64, device=device, generator=gen)])
    S = _structured_unitary_apply(torch.diag(sigma).to(dt), gen, req.cplx)
    H = _structured_unitary_apply(torch.diag(lam).to(dt), gen, req.cplx)
    S = 0.5 * (S + S.conj().T)
    H = 0.5 * (H + H.conj().T)
    return H.T.contiguous().T, S.T.contiguous().T


def scf_h(H0, req: Request, it: int):
    """H_t = H_0 + 1e-3 (G + G^H)/2, G seeded by (request, iteration)."""
    import torch

    gen = torch.Generator(device=H0.device)
    gen.manual_seed(req.seed * 101 + it + 1)
    n = H0.shape[0]
    g = torch.randn(n, n, dtype=torch.float64, device=H0.device, generator=gen)
    if H0.is_complex():
        g = (g + 1j * torch.randn(n, n, dtype=torch.float64, device=H0.device, generator=gen)) / math.sqrt(2.0)
    H = H0 + 1e-3 * 0.5 * (g + g.conj().T)
    return H.T.contiguous().T


class GpuWorkers:
    """Per-thread library handles, each with its own HIP stream."""

    def __init__(self, device, keep_results: bool = False):
        self.device = device
        self.keep = keep_results
        self.local = threading.local()
        self.results = {}
        self.rlock = threading.Lock()

    def _solver(self):
        import torch

        from . import gevd

        if not hasattr(self.local, "solver"):
            self.local.stream = torch.cuda.Stream(device=self.device)
            # several solves share the device: panels without co-residency
            self.local.solver = gevd.Solver(self.device, persistent_panel=False)
        return self.local.solver, self.local.stream

    def run_request(self, req: Request, on_solve, t0: float):
        import torch

        solver, stream = self._solver()
        with torch.cuda.stream(stream):
            H0, S = request_inputs(req, self.device)
            submit = req.arrival
            solver.set_overlap(S)
            outs = []
            for it in range(req.iters):
                H = scf_h(H0, req, it)
                w, C = solver.solve_resident(H, req.k)
                stream.synchronize()
                done = time.perf_counter() - t0
                on_solve(SolveRecord(req.rid, it, req.n, req.cplx, submit, done))
                if self.keep:
                    outs.append((w.cpu().numpy(), C.cpu().numpy()))
                submit = done
            del H0, S
        if self.keep:
            with self.rlock:
                self.results[req.rid] = outs

    def run_batch(self, reqs: list[Request], on_solve, t0: float):
        """Small requests together: the first SCF iteration factors every S
        in the batched kernel; the later ones replay a captured batch that
        reuses the factors (S fixed) with the iteration's H written into the
        same buffers."""
        import torch

        solver, stream = self._solver()
        with torch.cuda.stream(stream):
            outs, submits = batched_scf(solver, reqs, t0, on_solve, self.keep, stream)
        if self.keep:
            with self.rlock:
                self.results.update(outs)


def batched_scf(solver, reqs: list[Request], t0: float, on_solve=None, keep: bool = True, stream=None):
    """SCF iterations of a group of small requests on the batched path (the
    current stream).  Returns ({rid: [(eval, C) per iteration]}, last submit
    times)."""
    import torch

    inputs = [request_inputs(r, solver.device) for r in reqs]
    Hb = [torch.empty_like(H0) for H0, _ in inputs]
    Sb = [S.clone() for _, S in inputs]
    items = [(Hb[i], Sb[i], r.k) for i, r in enumerate(reqs)]
    outs = {r.rid: [] for r in reqs}
    submits = [r.arrival for r in reqs]
    its = max(r.iters for r in reqs)
    graph = None
    for it in range(its):
        for i, r in enumerate(reqs):
            Hb[i].copy_(scf_h(inputs[i][0], r, it))
        if it == 0:
            res, info = solver.solve_batched(items)
        else:
            if graph is None:
                graph = solver.batch(items, outs=res, factored=True)
            info = graph.run()
        if any(info):
            raise RuntimeError("batched solve failed: info %s" % info)
        (stream or torch.cuda.current_stream()).synchronize()
        done = time.perf_counter() - t0
        for i, r in enumerate(reqs):
            if it >= r.iters:
                continue
            if on_solve is not None:
                on_solve(SolveRecord(r.rid, it, r.n, r.cplx, submits[i], done, batched=True))
            submits[i] = done
            if keep:
                outs[r.rid].append((res[i][0].cpu().numpy(), res[i][1].cpu().numpy()))
    if graph is not None:
        graph.close()
    return outs, submits


def serve(requests: list[Request], device=None, budget_bytes: int | None = None, large_workers: int = 2,
          small_workers: int = 2, small_n: int = 512, batch: int = 8, batch_wait: float = 0.02,
          keep_results: bool = False, progress=None) -> StreamResult:
    """Serve a request stream on one GPU; returns per-solve records."""
    import torch

    from . import gevd

    device = torch.device(device or "cuda:0")
    torch.cuda.set_device(device)
    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info(device)
        budget_bytes = int(0.8 * free)
    workers = GpuWorkers(device, keep_results)

    def workspace_of(r: Request) -> int:
        return gevd.workspace_bytes(torch.complex128 if r.cplx else torch.float64, r.n, r.k)

    sched = Scheduler(budget_bytes, large_workers, small_workers, small_n, workspace_of, workers.run_request,
                      workers.run_batch, batch=batch, batch_wait=batch_wait, progress=progress)
    res = sched.run(requests)
    res.results = workers.results
    return res


def solve_alone(req: Request, device=None, small_n: int = 512):
    """The same request served by itself on the route the server gives it
    (a batch of one for n <= small_n, the resident path otherwise), with a
    fresh handle on the default stream."""
    import torch

    from . import gevd

    device = torch.device(device or "cuda:0")
    solver = gevd.Solver(device, persistent_panel=False)  # the server's panel route
    if req.n <= small_n:
        outs, _ = batched_scf(solver, [req], 0.0)
        solver.close()
        return outs[req.rid]
    H0, S = request_inputs(req, device)
    solver.set_overlap(S)
    outs = []
    for it in range(req.iters):
        w, C = solver.solve_resident(scf_h(H0, req, it), req.k)
        torch.cuda.synchronize()
        outs.append((w.cpu().numpy(), C.cpu().numpy()))
    solver.close()
    return outs


def batched_throughput(count: int = 1024, iters: int = 5, seed: int = 4, small=(64, 512), frac_complex: float = 0.6,
                       tune: bool = False, device=None) -> dict:
    """Throughput of the batched path alone on `count` small requests of the
    serving mix (n uniform in `small`, 60 % complex, lowest 30 %): the first
    SCF iteration factors every S; the later ones replay the captured batch
    with the factors reused.  Device time from the library's kernel
    accounting (HIP events around each launch)."""
    import torch

    from . import gevd

    device = torch.device(device or "cuda:0")
    torch.cuda.set_device(device)
    rng = np.random.default_rng(seed)
    reqs = []
    for rid in range(count):
        n = int(rng.integers(small[0], small[1] + 1))
        reqs.append(Request(rid, bool(rng.random() < frac_complex), n, max(1, int(math.ceil(0.3 * n - 1e-9))), 0.0,
                            seed=7_000_003 * seed + rid, iters=iters))
    solver = gevd.Solver(device, kstats=True)
    tuned = {}
    if tune:
        for dt in (torch.float64, torch.complex128):
            for nb in (64, 128, 256, 512):
                tuned["%s:%d" % ("z" if dt == torch.complex128 else "d", nb)] = solver.tune_batched(dt, nb, 512)
    inputs = [request_inputs(r, device) for r in reqs]
    Hb = [torch.empty_like(H0) for H0, _ in inputs]
    Sb = [S.clone() for _, S in inputs]
    items = [(Hb[i], Sb[i], r.k) for i, r in enumerate(reqs)]
    for i, r in enumerate(reqs):
        Hb[i].copy_(scf_h(inputs[i][0], r, 0))
    torch.cuda.synchronize()
    solver.reset_kernel_stats()
    t1 = time.perf_counter()
    res, info = solver.solve_batched(items)
    first_wall = time.perf_counter() - t1
    assert not any(info), info
    st = solver.kernel_stats()["small"]
    first = {"ms": st["ms"], "tflops": st["flops"] / (st["ms"] / 1e3) / 1e12}
    graph = solver.batch(items, outs=res, factored=True)
    solver.reset_kernel_stats()
    walls = []
    for it in range(1, iters):
        for i, r in enumerate(reqs):
            Hb[i].copy_(scf_h(inputs[i][0], r, it))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        info = graph.run()
        walls.append(time.perf_counter() - t1)
        assert not any(info), info
    st = solver.kernel_stats()["small"]
    later = {"ms_per_iter": st["ms"] / max(1, iters - 1), "tflops": st["flops"] / (st["ms"] / 1e3) / 1e12}
    graph.close()
    shapes = {"%s:%d" % (tag, nb): solver.batch_shape(dt, nb) for dt, tag in ((torch.float64, "d"),
                                                                             (torch.complex128, "z"))
              for nb in (64, 128, 256, 512)}
    solver.close()
    return {"mode": "batched", "problems": count, "complex_fraction": frac_complex, "n_range": list(small),
            "first_iteration": {"device_ms": round(first["ms"], 2), "wall_ms": round(first_wall * 1e3, 2),
                                "solves_per_s": round(count / (first["ms"] / 1e3), 1),
                                "tflops": round(first["tflops"], 3)},
            "factored_iterations": {"device_ms": round(later["ms_per_iter"], 2),
                                    "wall_ms": round(1e3 * float(np.median(walls)), 2) if walls else None,
                                    "solves_per_s": round(count / (later["ms_per_iter"] / 1e3), 1),
                                    "tflops": round(later["tflops"], 3)},
            "shapes": shapes, "tuned": tuned}


def main():
    import argparse
    import json

    ap = argparse.ArgumentParser(description="serve a Poisson stream of generalized eigensolves")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--iters", type=int, default=5)
    ap.add_argument("--large-max", type=int, default=8192)
    ap.add_argument("--large-workers", type=int, default=2)
    ap.add_argument("--small-workers", type=int, default=2)
    ap.add_argument("--mode", choices=("stream", "batched"), default="stream")
    ap.add_argument("--tune", action="store_true", help="batched mode: run the shape tuner first")
    args = ap.parse_args()
    if args.mode == "batched":
        print(json.dumps(batched_throughput(args.requests, args.iters, tune=args.tune)), flush=True)
        return
    reqs = poisson_stream(args.requests, args.rate, large=(1024, args.large_max), iters=args.iters)
    def progress(done, total, secs):
        print("served %d/%d requests at %.1f s" % (done, total, secs), file=sys.stderr, flush=True)

    res = serve(reqs, large_workers=args.large_workers, small_workers=args.small_workers, progress=progress)
    out = res.summary()
    out.update({"requests": args.requests, "rate_per_s": args.rate, "iters": args.iters,
                "error_messages": [m for _, m in res.errors][:4]})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
