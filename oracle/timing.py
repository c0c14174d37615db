"""Times the CPU oracle on a bounded sample of a workload (test
infrastructure: run by the benchmark's CPU-baseline leg only).

    python -m oracle.timing --config 2 --theta 0.3 --p 10 --leaf-fraction 64 --runs 10

The sample is every particle of a seeded random subset of the tree's leaves
(1/leaf_fraction of them), evaluated by the oracle's FMM as targets: one call
is the full upward pass (P2M, M2M over every cell), the M2L, L2L and L2P of
the sampled leaves and their ancestors, and their near field.  Run the
process with the OpenMP placement wanted (OMP_NUM_THREADS, OMP_PROC_BIND,
OMP_PLACES, OMP_WAIT_POLICY), which the runtime reads once at start-up.
Prints one JSON line: per-run seconds, their median, the targets evaluated
per run and the threads used.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--leaf-fraction", type=int, default=64, help="evaluate 1 in this many leaves")
    ap.add_argument("--runs", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--method", choices=["fmm", "bh"], default="fmm")
    a = ap.parse_args()

    import oracle
    from paper_2005_12351_amd import workloads as W

    w = W.config(a.config)
    theta = w.theta if a.theta is None else a.theta
    p = w.p if a.p is None else a.p
    t = oracle.Tree(w.pos, w.ncrit, theta if a.method == "fmm" else None)
    d = t.dump()
    leaves = np.nonzero(d.nchild == 0)[0]
    rng = np.random.default_rng(20051235)
    k = max(1, len(leaves) // a.leaf_fraction)
    pick = np.sort(rng.choice(leaves, size=k, replace=False))
    tg = np.sort(np.concatenate([d.perm[d.first[c]:d.first[c] + d.count[c]] for c in pick])).astype(np.int64)

    def once():
        if a.method == "fmm":
            t.fmm(w.order, w.moments, p, targets=tg)
        else:
            t.bh(w.order, w.moments, p, theta, targets=tg)

    for _ in range(a.warmup):
        once()
    secs = []
    for _ in range(a.runs):
        t0 = time.perf_counter()
        once()
        secs.append(time.perf_counter() - t0)
    print(json.dumps({"seconds": secs, "median_s": float(np.median(secs)), "targets": int(tg.shape[0]),
                      "leaves": int(k), "leaves_total": int(len(leaves)), "n": w.n, "theta": theta, "p": p,
                      "threads": int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count(),
                      "method": a.method}), flush=True)


if __name__ == "__main__":
    main()
