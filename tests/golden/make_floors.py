"""Writes tests/golden/floors.json: the FP64 floor F (tests/floors.py) of
every whole-solve parity input, from the CPU oracle alone.

    python tests/golden/make_floors.py            # all cases (c1 takes minutes)
    python tests/golden/make_floors.py --small    # without the n = 4096 case

Each entry: {"F": max relative spread over the k wanted, "F_normwise": the
same normwise over all n}, from two perturbation draws.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from tests import cases, floors  # noqa: E402


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--small", action="store_true", help="skip the full-size configuration")
    a = ap.parse_args()
    old = {}
    if os.path.exists(floors.GOLDEN):
        with open(floors.GOLDEN) as f:
            old = json.load(f).get("floors", {})
    out = dict(old)
    for key, H, S, k, nh, ns in cases.all_cases(include_large=not a.small):
        t = time.time()
        out[key] = floors.floor(H, S, k, norm_h=nh, norm_s=ns)
        print("%-60s F %.3e  normwise %.3e  (%.1f s)" % (key, out[key]["F"], out[key]["F_normwise"],
                                                        time.time() - t), flush=True)
    doc = {"what": "FP64 floor of each parity input: oracle eigenvalue spread under u-sized Hermitian "
                   "perturbations of H and S (tests/floors.py)",
           "command": "python tests/golden/make_floors.py",
           "oracle_threads": oracle.threads(),
           "floors": dict(sorted(out.items()))}
    tmp = floors.GOLDEN + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, floors.GOLDEN)
    return 0


if __name__ == "__main__":
    sys.exit(main())
