"""Benchmark: dense generalized Hermitian eigensolve H c = eps S c on one GPU.

A step is one whole solve (Cholesky, inversion, the two products, full ->
band, band -> tridiagonal, divide-and-conquer, the three back-
transformations) of a freshly copied input pair already resident in HBM.
Default workload: complex Hermitian n = 16384, lowest 25 % of eigenpairs,
overlap condition number ~1e6 (synthetic DFT-shaped pencil, drawn on the
device).  Prints ONE JSON line.

The metric is the solve's nominal throughput: F_nom / time with
F_nom = 8 n^3/3 + 5 n^2 k real flops (x4 for complex): Cholesky n^3/3,
reduction n^3, full -> band 4n^3/3, the two reflector back-transformations
2 n^2 k each and C = U^{-1} C~ n^2 k.  Bulge chasing and divide-and-conquer
are excluded from the numerator (timed, not counted).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    # name: (n, complex, sigma_min, frac, seed, label)
    "c0": (256, False, 1e-3, 1.0, 0, "real symmetric n=256, all pairs, kappa(S)~1e3"),
    "c1": (4096, False, 1e-6, 0.30, 1, "real symmetric n=4096, lowest 30%, kappa(S)~1e6"),
    "c2": (16384, True, 1e-6, 0.25, 2, "complex Hermitian n=16384, lowest 25%, kappa(S)~1e6"),
    "c3": (8192, False, 1e-6, 0.30, 3, "real symmetric n=8192, lowest 30%, kappa(S)~1e6"),
}

FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak (datasheet); the FP64 vector peak is the same
# roofline bound of each kernel family: the products (GEMM and the stage-2
# back-transformation's block products) against the FP64 matrix peak; the
# panel, bulge-chasing, D&C and small-solve kernels are latency/ALU-bound
FAMILY_BOUND = {"gemm": "mfma", "gemm32": "mfma", "backchase": "mfma", "panel": "alu", "chase": "alu", "dc": "alu",
                "other": "alu", "small": "alu"}


def nominal_flops(n: int, k: int, cplx: bool) -> float:
    f = 8.0 * n ** 3 / 3.0 + 5.0 * n * n * k
    return 4.0 * f if cplx else f


def method_flops(n: int, k: int, cplx: bool) -> dict:
    """The nominal flops each kernel family carries (real count, x4
    complex): the GEMM family does the Cholesky updates (n^3/3), the
    reduction (n^3), full -> band (4n^3/3), the stage-1 back-transformation
    (2n^2 k) and C = U^{-1} C~ (n^2 k); the stage-2 back-transformation
    kernel does 2n^2 k.  Work a route executes beyond these (the explicit
    inverse, the second reduction product, divide-and-conquer merges) is
    not credited: it is in the families' executed-flop rates instead."""
    c = 4.0 if cplx else 1.0
    return {"gemm": c * (n ** 3 / 3.0 + n ** 3 + 4.0 * n ** 3 / 3.0 + 3.0 * n * n * k),
            "backchase": c * 2.0 * n * n * k}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def measured_traffic(config: str, family: str, band: int):
    """HBM bytes per launch of a kernel family from the committed PMC
    summary (profiles/), or None when there is none for this workload and
    band width, or the kernel's source or a caller that fixes its launch
    shapes changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "%s_family_%s_traffic.json" % (family, config))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("band") != band:
        return None
    # the kernel's source and its callers' (which fix the launch shapes)
    for rel, sha in rec["sources"].items():
        src = os.path.join(ROOT, rel)
        if not os.path.exists(src):
            return None
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != sha:
                return None
    return rec["hbm_bytes_per_launch"]


def plain_inputs(n: int, cplx: bool, frac: float, seed: int, dev):
    """H = (G + G^H)/2 with G Gaussian, S = I + (R + R^H)/(4n): elementwise
    device ops only."""
    import torch

    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    dt = torch.complex128 if cplx else torch.float64

    def draw():
        x = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
        if cplx:
            x = torch.complex(x, torch.randn(n, n, dtype=torch.float64, device=dev, generator=g))
        return x

    G = draw()
    H = (0.5 * (G + G.mT.conj())).to(dt)
    del G
    R = draw()
    S = ((R + R.mT.conj()) / (4.0 * n)).to(dt)
    del R
    S.diagonal().add_(1.0)
    k = max(1, int(math.ceil(frac * n - 1e-9)))
    return H.mT.contiguous().mT, S.mT.contiguous().mT, k


def _norm2_est(M, iters: int = 30) -> float:
    """2-norm of a Hermitian device matrix by power iteration."""
    import torch

    g = torch.Generator(device=M.device)
    g.manual_seed(5)
    x = torch.randn(M.shape[0], dtype=torch.float64, device=M.device, generator=g).to(M.dtype)
    x = x / torch.linalg.vector_norm(x)
    nrm = 0.0
    for _ in range(iters):
        y = M @ x
        nrm = float(torch.linalg.vector_norm(y))
        x = y / nrm
    return nrm


def sample_eta(H, S, w, C, k, count: int = 8, norms=None):
    """Backward error eta_i = ||H c - w S c|| / ((||H|| + |w| ||S||) ||c||)
    for `count` wanted pairs spread over the k (device products, FP64)."""
    import torch

    nh, ns = norms if norms is not None else (_norm2_est(H), _norm2_est(S))
    idx = sorted(set(int(round(i * (k - 1) / max(count - 1, 1))) for i in range(count)))
    Cs = C[:, idx]
    R = H @ Cs - (S @ Cs) * w[idx].to(C.dtype)[None, :]
    eta = torch.linalg.vector_norm(R, dim=0) / ((nh + w[idx].abs() * ns) * torch.linalg.vector_norm(Cs, dim=0))
    return float(eta.max()), (nh, ns)


def cpu_baseline(cplx: bool, n_full: int, k_frac: float, sigma_min: float, budget_s: float = 20.0):
    """The oracle, as it stands, on a bounded sample of the same workload:
    the same recipe at the largest n whose oracle solve fits the time budget,
    scaled to the full n by the n^3 cost law."""
    import numpy as np

    import oracle
    from paper_2502_02460_amd import synth

    n = 256
    last = None
    while True:
        p = synth.pencil(n, cplx, sigma_min, 99, k_frac)
        t0 = time.perf_counter()
        oracle.gevd(p.H, p.S, p.k)
        dt = time.perf_counter() - t0
        last = (n, p.k, dt)
        if dt * 8.5 > budget_s or n * 2 > n_full:
            break
        n *= 2
    n, k, dt = last
    rate = nominal_flops(n, k, cplx) / dt / 1e12
    t_full = dt * (n_full / n) ** 3
    return {"value": rate, "unit": "TFLOP/s", "cores": oracle.threads(), "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "oracle solve of the same recipe at n=%d (k=%d) took %.2f s; extrapolated n=%d solve %.0f s" %
                      (n, k, dt, n_full, t_full)}


def serving_legs(args, dev) -> dict:
    """The batched path on a batch of the serving mix's small problems, and
    a labelled serving stream of the c4 size mix (70 % n in [64, 512]
    batched, 30 % n in [1024, 8192] resident; 60 % complex; lowest 30 %;
    five SCF iterations per request with S fixed) at an arrival rate that
    keeps one GPU at about 70 % utilisation.  The stream as specified (2048
    requests at 200 per second, about 7x one GPU's FP64 peak) is a
    saturation test that would run for tens of minutes."""
    import torch

    from paper_2502_02460_amd import serve

    torch.cuda.empty_cache()
    t1 = time.time()
    bt = serve.batched_throughput(count=args.batch_problems, iters=3, device=dev)
    print("# batched leg: %d problems in %.1f s" % (args.batch_problems, time.time() - t1), file=sys.stderr,
          flush=True)
    reqs = serve.poisson_stream(args.serve_requests, args.serve_rate, iters=5)

    def progress(done, total, secs):
        print("# serving leg: %d/%d requests done at %.1f s" % (done, total, secs), file=sys.stderr, flush=True)

    t1 = time.time()
    res = serve.serve(reqs, device=dev, large_workers=2, small_workers=2, progress=progress)
    summ = res.summary()
    print("# serving leg: %.1f s" % (time.time() - t1), file=sys.stderr, flush=True)
    rnd = {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in summ.items()}
    rnd["by_class"] = {c: {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in d.items()}
                       for c, d in summ["by_class"].items()}
    return {"batched": bt,
            "serving": {"label": "c4 size mix, %d requests x 5 SCF iterations, Poisson %.2f requests/s "
                                 "(about 70%% utilisation of one GPU)" % (args.serve_requests, args.serve_rate),
                        "requests": args.serve_requests, "rate_per_s": args.serve_rate, **rnd}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--band", type=int, default=0)
    ap.add_argument("--stages", type=int, default=2, choices=(1, 2),
                    help="tridiagonalisation: 2 = full -> band -> tridiagonal, 1 = one-stage Householder")
    ap.add_argument("--frac", type=float, default=None, help="override the wanted fraction (1.0 = all pairs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32+refine comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the batched and serving legs")
    ap.add_argument("--batch-problems", type=int, default=512,
                    help="batched leg: small problems of the serving mix (n in [64, 512], 60%% complex)")
    ap.add_argument("--serve-requests", type=int, default=40, help="serving leg: requests in the stream")
    ap.add_argument("--serve-rate", type=float, default=1.2,
                    help="serving leg: mean arrivals per second (about 70%% of one GPU's capacity for the mix)")
    ap.add_argument("--inputs", choices=("paper", "plain"), default="paper",
                    help="plain: H random Hermitian, S = I + R/(4n), drawn with elementwise device ops only "
                         "(no library QR or BLAS calls; for profiler passes that cannot instrument those)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2502_02460_amd import gevd, synth

    n, cplx, smin, frac, seed, label = CONFIGS[args.config]
    if args.frac is not None:
        frac = args.frac
        label = label.split(",")[0] + ", wanted fraction %g" % frac + "," + ",".join(label.split(",")[2:])
    if args.stages == 1:
        label += ", one-stage tridiagonalisation"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    if args.inputs == "paper":
        H0, S0, k, _ = synth.pencil_torch(n, cplx, smin, seed, frac, dev)
    else:
        H0, S0, k = plain_inputs(n, cplx, frac, seed, dev)
    torch.cuda.synchronize()
    print("# inputs drawn in %.1f s (n=%d k=%d %s)" % (time.time() - t0, n, k, "complex" if cplx else "real"),
          file=sys.stderr, flush=True)
    # the timed steps run without per-launch events; one more step with the
    # kernel-family accounting on gives the roofline figures
    solver = gevd.Solver(dev, band=args.band, timing=True, kstats=False, stages=args.stages)
    H = torch.empty_like(H0)
    S = torch.empty_like(S0)
    C = torch.empty((k, n), dtype=H0.dtype, device=dev).mT
    w = torch.empty(n, dtype=torch.float64, device=dev)

    work_stream = torch.cuda.Stream(device=dev)  # a non-default stream (default priority)

    def step():
        with torch.cuda.stream(work_stream):
            H.copy_(H0)
            S.copy_(S0)
            solver.solve(H, S, k, C=C, eval_out=w)

    for i in range(args.warmup):
        t1 = time.time()
        step()
        torch.cuda.synchronize()
        print("# warmup %d: %.3f s" % (i, time.time() - t1), file=sys.stderr, flush=True)
    per = []
    phases = []
    torch.cuda.synchronize()
    solver.reset_kernel_stats()
    tstart = time.perf_counter()
    for i in range(args.steps):
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        per.append(time.perf_counter() - t1)
        phases.append(solver.timings())
        print("# step %d: %.3f s" % (i, per[-1]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - tstart
    solver.set_kstats(True)
    step()
    torch.cuda.synchronize()
    ks = solver.kernel_stats()
    solver.set_kstats(False)
    kstat_steps = 1
    ms = 1e3 * total / args.steps
    fl = nominal_flops(n, k, cplx)
    value = fl / (total / args.steps) / 1e12
    sp = sorted(per)
    p50 = sp[len(sp) // 2] if len(sp) % 2 else 0.5 * (sp[len(sp) // 2 - 1] + sp[len(sp) // 2])
    p99 = sp[min(len(sp) - 1, int(math.ceil(0.99 * len(sp))) - 1)]
    ph = {kk: sum(p[kk] for p in phases) / len(phases) for kk in phases[0]}
    red_fl = (4.0 if cplx else 1.0) * (n ** 3 / 3.0 + n ** 3 + 4.0 * n ** 3 / 3.0)
    red_ms = ph["cholesky"] + ph["invert"] + ph["multiply"] + ph["band"]
    # accuracy of the last step on the commuting-free pencil: S-orthonormality
    # and backward error of a sample of eigenpairs (device products)
    out = {
        "metric": "n=%d gen. eigensolve TFLOP/s (FP64)" % n,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if cplx else "f64",
        "data": "synthetic",
        "config": {"workload": label if args.inputs == "paper" else label + " (plain inputs)", "n": n, "nev": k,
                   "complex": cplx, "sigma_min": smin, "stages": args.stages,
                   "band": solver.band_width(n, H0.dtype) if args.stages == 2 else None},
        "p50_s": round(p50, 4),
        "p99_s": round(p99, 4),
        "phases_ms": {kk: round(v, 2) for kk, v in ph.items()},
        "reduction_phases_tflops": round(red_fl / (red_ms / 1e3) / 1e12, 3),
        "reduction_phases_frac_fp64_peak": round(red_fl / (red_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS, 4),
    }
    fams = {k: v for k, v in ks.items() if v["launches"] > 0}
    mfl = method_flops(n, k, cplx)
    out["kernels"] = {}
    for kk, v in fams.items():
        rec = {"launches": v["launches"] // kstat_steps, "ms_per_step": round(v["ms"] / kstat_steps, 2),
               "executed_tflops": round(v["flops"] / (v["ms"] / 1e3) / 1e12, 3) if v["ms"] > 0 else None}
        if kk in mfl and v["ms"] > 0:
            rec["method_tflops"] = round(mfl[kk] / (v["ms"] / 1e3 / kstat_steps) / 1e12, 3)
        out["kernels"][kk] = rec
    dom = max(fams, key=lambda kk: fams[kk]["ms"])
    g = fams[dom]
    # achieved: the method's flops this family carries (not what the route
    # executes) per step over the family's device time per step
    ach = (mfl.get(dom, 0.0) / (g["ms"] / 1e3 / kstat_steps) / 1e12) if g["ms"] > 0 else 0.0
    out["roofline"] = {"kernel": dom, "bound": FAMILY_BOUND[dom], "achieved": round(ach, 3),
                       "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4),
                       "traffic": measured_traffic(args.config, dom, solver.band_width(n, H0.dtype)),
                       "launches_per_step": g["launches"] // kstat_steps,
                       "avg_launch_ms": round(g["ms"] / g["launches"], 4),
                       "method_tflop_per_step": round(mfl.get(dom, 0.0) / 1e12, 3),
                       "executed_tflops": round(g["flops"] / (g["ms"] / 1e3) / 1e12, 3)}
    if not args.no_fp32:
        # the same workload in the reduced-precision form, compared with the
        # FP64 result of the last timed step on the same input
        w64 = w.clone()
        C64 = C.clone()
        eta64, norms = sample_eta(H0, S0, w64, C64, k)
        solver.set_precision("fp32+refine", 2)
        for i in range(args.warmup):
            step()
        torch.cuda.synchronize()
        per32 = []
        t32 = time.perf_counter()
        for i in range(args.steps):
            t1 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            per32.append(time.perf_counter() - t1)
            print("# fp32+refine step %d: %.3f s" % (i, per32[-1]), file=sys.stderr, flush=True)
        tot32 = time.perf_counter() - t32
        eta32, _ = sample_eta(H0, S0, w, C, k, norms=norms)
        nrm = float(w64[:k].abs().max())
        sp = sorted(per32)
        out["fp32_refine"] = {
            "ms_per_step": round(1e3 * tot32 / args.steps, 2),
            "value": round(fl / (tot32 / args.steps) / 1e12, 3),
            "p50_s": round(sp[len(sp) // 2], 4), "p99_s": round(sp[-1], 4),
            "speedup_vs_fp64": round((total / args.steps) / (tot32 / args.steps), 3),
            "eig_err_vs_fp64_normwise": float((w[:k] - w64[:k]).abs().max()) / nrm,
            "eta_sample_max": eta32, "eta_sample_max_fp64": eta64,
            "refine_sweeps": 2,
        }
        solver.set_precision("fp64")
    solver.close()
    if not args.no_serving:
        out.update(serving_legs(args, dev))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cplx, n, frac, smin)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
