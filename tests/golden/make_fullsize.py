"""Writes tests/golden/fullsize_oracle.json: the CPU oracle's own accuracy on
the full-size commuting pencils that tests/test_gpu_fullsize.py solves on
the GPU (real n = 4096 and 8192, lowest 30 %, kappa(S) ~ 1e6).

The inputs are drawn with synth.pinned_problem (fixed OpenBLAS kernel type
and thread count, so the same bits on any AVX2 host; each entry records the
input's SHA-256).  For each: the oracle's whole solve, its normwise error
against the exact spectrum lam_i / sigma_i over all n eigenvalues, its
backward errors at the columns the GPU test samples and over all k wanted
columns, and its S-orthonormality.  The GPU test holds the solver to
max(1e-11, 2x) these values on the same input.

    python tests/golden/make_fullsize.py            # minutes (n = 8192: ~30 min on 8 cores)
    python tests/golden/make_fullsize.py --floors   # adds each input's FP64 floor (tests/floors.py)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2502_02460_amd import synth  # noqa: E402
from tests import floors  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_oracle.json")
# (n, seed) of the real commuting full-size cases; lowest 30 %, sigma_min 1e-6
CASES = [(4096, 31), (8192, 33)]
SAMPLES = 8


def sample_index(k: int, count: int = SAMPLES) -> list:
    """Columns spread evenly over the k wanted (the GPU test samples these)."""
    return sorted(set(int(round(i * (k - 1) / (count - 1))) for i in range(count)))


def key(n: int, seed: int) -> str:
    return "commuting/n=%d/d/smin=1e-06/seed=%d/f=0.3" % (n, seed)


def main() -> int:
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f).get("cases", {})
    only = [int(a) for a in sys.argv[1:] if a != "--floors"]
    floors_only = "--floors" in sys.argv[1:]
    for n, seed in CASES:
        if only and n not in only:
            continue
        t = time.time()
        p, sha = synth.pinned_problem("commuting", n, False, 1e-6, seed, 0.3)
        if floors_only and key(n, seed) in out:
            # the input's FP64 floor (tests/floors.py) on top of the stored entry
            fl = floors.floor(p.H, p.S, p.k, norm_h=float(abs(p.lam).max()), norm_s=float(p.sigma.max()))
            out[key(n, seed)].update({"F": fl["F"], "F_normwise": fl["F_normwise"]})
            print(key(n, seed), fl, flush=True)
            doc = {"what": "CPU oracle accuracy on the full-size commuting pencils (tests/golden/make_fullsize.py)",
                   "command": "python tests/golden/make_fullsize.py; python tests/golden/make_fullsize.py --floors",
                   "cases": out}
            with open(OUT + ".tmp", "w") as f:
                json.dump(doc, f, indent=1)
            os.replace(OUT + ".tmp", OUT)
            continue
        w, C, _ = oracle.gevd(p.H, p.S, p.k)
        nh, ns = float(np.abs(p.lam).max()), float(p.sigma.max())
        R = p.H @ C - (p.S @ C) * w[None, : p.k]
        eta = np.linalg.norm(R, axis=0) / ((nh + np.abs(w[: p.k]) * ns) * np.linalg.norm(C, axis=0))
        idx = sample_index(p.k)
        Cs = C[:, idx]
        orth = float(np.abs(Cs.T @ (p.S @ Cs) - np.eye(len(idx))).max())
        err = float(np.abs(w - p.exact).max() / np.abs(p.exact).max())
        out[key(n, seed)] = {"sha256": sha, "k": p.k, "sample_index": idx,
                             "eta_sampled": [float(eta[i]) for i in idx], "eta_max_all": float(eta.max()),
                             "eig_err_normwise": err,
                             "eig_rel_wanted": float((np.abs(w[: p.k] - p.exact[: p.k]) / np.abs(p.exact[: p.k])).max()),
                             "orth_sampled": orth, "oracle_threads": oracle.threads(),
                             "oracle_seconds": round(time.time() - t, 1)}
        print(key(n, seed), json.dumps(out[key(n, seed)]), flush=True)
        doc = {"what": "CPU oracle accuracy on the full-size commuting pencils (tests/golden/make_fullsize.py)",
               "command": "python tests/golden/make_fullsize.py; python tests/golden/make_fullsize.py --floors",
               "cases": out}
        with open(OUT + ".tmp", "w") as f:
            json.dump(doc, f, indent=1)
        os.replace(OUT + ".tmp", OUT)
    return 0


if __name__ == "__main__":
    sys.exit(main())
