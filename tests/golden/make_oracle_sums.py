#!/usr/bin/env python3
"""Writes the FP64 oracle's path sums at full benchmark sizes.

Calls only ``oracle/`` (and the input generators in ``workloads``): the HIP
library is never loaded here.  Each file holds, per scheme, the oracle's sums
of the caplet payoffs of eq. (caplet) (Section 3.3) over consecutive chunks of
paths -- sum p, sum p^2, in-the-money counts per (caplet, strike); sum M and
sum M^2 of the martingale factor M = prod_{l>=i}(1 + delta_l L_l) -- on the
Philox streams of seed 1, tag 0.  The GPU tests add the chunks up (in chunk
order) and compare prices per caplet; a CPU test recomputes one chunk.

    python tests/golden/make_oracle_sums.py [c2|c4|all]

C2 (N = 20, 400 steps, 2^20 paths, FULL and PICARD) takes ~7 min on 8 cores,
C4 (N = 40, 400 steps, 2^16 paths, FULL, PICARD, FIRST_ORDER, SECOND_ORDER)
~2.5 min.  The oracle runs with THREADS OpenMP threads; its sum order inside a
chunk depends on that count, so the recheck uses the same count.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

THREADS = 8
SCHEME_IDS = {"full": oracle.FULL, "picard": oracle.PICARD, "first_order": oracle.FIRST_ORDER,
              "second_order": oracle.SECOND_ORDER}
FILES = {
    "c2": ("oracle_sums_gpu_n20_2p20.json", workloads.gpu_scale, 1 << 20, 1 << 16,
           ("full", "picard")),
    "c4": ("oracle_sums_mlp_n40_2p16.json", workloads.learned_drift, 1 << 16, 1 << 14,
           ("full", "picard", "first_order", "second_order")),
}
KEYS = ("sum_p", "sum_p2", "n_itm", "sum_mart", "sum_mart2")


def chunk_sums(o, scheme: str, p0: int, n: int) -> dict:
    r = o.price_sums(SCHEME_IDS[scheme], n, path0=p0, threads=THREADS)
    return {k: r[k].tolist() for k in KEYS}


def write(which: str) -> str:
    fname, make, n_paths, chunk, schemes = FILES[which]
    ts = make()
    o = oracle.Oracle(ts, seed=1)
    out = {"workload": ts.name, "seed": 1, "n_paths": n_paths, "chunk_paths": chunk,
           "threads": THREADS, "n_rates": ts.n_rates, "n_strikes": ts.n_strikes,
           "stat_keys": list(KEYS), "schemes": {}}
    for name in schemes:
        t0 = time.perf_counter()
        out["schemes"][name] = [chunk_sums(o, name, p0, chunk) for p0 in range(0, n_paths, chunk)]
        print(f"{which} {name}: {time.perf_counter() - t0:.1f} s", flush=True)
    path = os.path.join(HERE, fname)
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    return path


if __name__ == "__main__":
    arg = sys.argv[1] if len(sys.argv) > 1 else "all"
    oracle.build(force=False)
    for w in (("c2", "c4") if arg == "all" else (arg,)):
        print(write(w), flush=True)
