"""Benchmark of the sampled temporal-motif counting path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = one pass of the whole path over one synthetic graph already in
HBM: load (validate, normalise, radix sort, incidence lists), exact counts
of the workload's motifs, and its estimates (window partition, Philox
sampling, per-window exact counts, FP64 weighting).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import tm_inputs as ti  # noqa: E402

WORKLOADS = {
    # name: (graph factory, motifs, delta, [(c, p)], description)
    "small": (ti.config_small, [ti.TRIANGLE], 3600, [(30, 0.1)],
              "1k nodes, 20k uniform edges over [0,1e6), triangle, delta 3600, c 30, p 0.1"),
    "small_dense": (ti.config_small_dense, [ti.TRIANGLE], 3600, [(30, 0.1)],
                    "50 nodes, 20k uniform edges over [0,1e6), triangle, delta 3600, c 30, p 0.1"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="small")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding is a design "
              "note, not an implemented path", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1810_00980_amd as tm

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    fac, motifs, delta, est, desc = WORKLOADS[args.workload]
    log("generating", args.workload)
    g = fac()
    src, dst, t = (torch.from_numpy(a).cuda() for a in (g.src, g.dst, g.t))
    torch.cuda.synchronize()

    def step():
        G = tm.load_graph(src, dst, t, g.n)
        exact = tm.count_exact_multi(G, motifs, delta)
        ests = []
        for (c, p) in est:
            z, _ = tm.estimate_multi(G, motifs, delta, c, p, 0)
            ests.append(z)
        G.free()
        return exact, ests

    for i in range(args.warmup):
        step()
        log("warmup", i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        exact, ests = step()
        log("step", i)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    q = len(motifs) * (1 + len(est))
    value = g.m * q / dt
    out = {
        "metric": "temporal edges/s per motif query (exact & p=0.1 estimate)",
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": desc, "m": g.m, "n": g.n, "queries_per_step": q},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
