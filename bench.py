"""Benchmark of the sampled temporal-motif counting path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step is one pass of the whole path over one synthetic temporal graph
whose arrays are already in HBM:
  load       validate ids, normalise times, radix-sort by time, build the
             per-node incidence lists and pair indexes;
  exact      exact counts of every motif of the workload (one sweep);
  estimates  for each (c, p) of the workload and every motif: shift draw,
             window partition, Philox window sampling, exact counts of the
             kept windows and the weighted sum (one sweep per (c, p));
then the graph is freed.  Prints one JSON line on stdout.

value = temporal edges x motif queries answered per step / seconds per step
(a motif query is one motif's exact count or one motif's estimate at one
(c, p)).  The roofline object reports the dominant sweep kernel (the one
with the most time per step when each kernel of a pass runs alone): its HBM
traffic per launch, from the committed rocprofv3 FETCH_SIZE + WRITE_SIZE
record of the current kernel source (calibrated by a plain copy), over its
average launch time measured with HIP events on the launch stream inside the
library, against 8 TB/s; and beside it the algorithmic bytes per launch of
the work census with the per-unit figures of the method (16 B per anchor,
12 B per scanned list entry, 8 B per binary-search probe, 8 B per weight
read).

Profiling helpers (rocprofv3 -f csv output directories):
  --profile-run                 only the serial-timing step and one timed
                                step (for rocprofv3 runs)
  --pmc-summary FETCH WRITE     write profiles/<kernel>_zipf10m_traffic.json
  --kt-summary DIR              write profiles/sweep3_zipf10m_kernel_trace.txt
  --pmc-counters DIR            write profiles/sweep3_zipf10m_counters.json
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import tm_inputs as ti  # noqa: E402

THREE = ti.three_edge_motifs()
HBM_PEAK_GBS = 8000.0
# library timing names of the three-edge sweep kernels (exact, then weighted)
SWEEP_KERNELS = ("sweep3_fwd_count", "sweep3_tri_count", "sweep3_bwd_count",
                 "sweep3_fwd_weight", "sweep3_tri_weight", "sweep3_bwd_weight",
                 "tri_static_weight", "tri_static_prep")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1810_00980_amd", "csrc", f)
               for f in ("tm_sweep3.hip", "tm_sweep_dev.h", "tm_common.h", "tm_tri_static.hip")]

WORKLOADS = {
    "zipf10m": dict(
        graph=ti.config_zipf10m, motifs=THREE, delta=3600,
        est=[(10, 0.01), (10, 0.1), (30, 0.01), (30, 0.1)],
        desc="100k nodes, 10M edges, Zipf(1.8) endpoints, bursty Poisson times over [0,3e7) s; "
             "all 36 three-edge motifs (32 three-node + 4 two-node), delta 3600; exact + estimates "
             "at c in {10,30} x p in {0.01,0.1}, seed 0"),
    "small": dict(
        graph=ti.config_small, motifs=[ti.TRIANGLE], delta=3600, est=[(30, 0.1)],
        desc="1k nodes, 20k uniform edges over [0,1e6), triangle, delta 3600, c 30, p 0.1, seed 0"),
    "small_dense": dict(
        graph=ti.config_small_dense, motifs=[ti.TRIANGLE], delta=3600, est=[(30, 0.1)],
        desc="50 nodes, 20k uniform edges over [0,1e6), triangle, delta 3600, c 30, p 0.1, seed 0"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, motifs, delta, frac=0.03):
    """The oracle's indexed tier (every first/last edge pair sharing a node
    within delta, middles by range counts; OpenMP over anchors) timed on the
    host cores, single-threaded and with every core, on a bounded sample of
    the same workload: the exact counts of all the step's motifs on the
    sub-graph of the edges in the first `frac` of the time span (a contiguous
    slice at the workload's own density and burstiness).  Rate = slice edges
    x motifs / seconds, the unit of the GPU's value."""
    import oracle
    hi = int(g.t.min() + frac * (int(g.t.max()) - int(g.t.min())))
    sel = g.t < hi
    s, d, t = g.src[sel], g.dst[sel], g.t[sel]
    oracle.count3_indexed(s[:1000], d[:1000], t[:1000], motifs, delta, threads=1)  # load, build
    cores = os.cpu_count() or 1
    out = {}
    for threads in (1, cores):
        t0 = time.perf_counter()
        oracle.count3_indexed(s, d, t, motifs, delta, threads=threads)
        out[threads] = time.perf_counter() - t0
    m = int(sel.sum())
    return {"value": m * len(motifs) / out[cores], "unit": "edges/s", "cores": cores, "kind": "oracle",
            "single_thread_value": m * len(motifs) / out[1], "single_thread_s": out[1], "all_cores_s": out[cores],
            "host_cpu": _host_cpu_model(),
            "sample": f"exact counts of all {len(motifs)} motifs on the {m} edges of the first {frac:.0%} of the "
                      f"time span (a contiguous slice of the same graph), oracle tier C (indexed: first/last "
                      f"edge pairs sharing a node, middles by range counts), {cores} host threads and 1 thread"}


def run_batch(args):
    """Batched estimator on the 50M-edge workload: 64 seeds of the triangle
    estimate (delta 3600, c 30, p 0.1) per launch sequence.  A timed step is
    cold: the graph's cached batch state is released first, so the step
    includes building the stored anchor values, capturing the hipGraph and
    the run.  Warm replays (new seeds, cached state) and the same 64
    estimates one call at a time are reported beside it, with the mean and
    variance of the 64 estimates against the exact count."""
    import torch
    import paper_1810_00980_amd as tm
    delta, c, p, M = 3600, 30, 0.1, ti.TRIANGLE
    log("generating batch50m")
    g = ti.config_batch50m()
    src, dst, t = (torch.from_numpy(a).cuda() for a in (g.src, g.dst, g.t))
    torch.cuda.synchronize()
    G = tm.load_graph(src, dst, t, g.n)
    L = c * delta
    win = np.bincount((g.t - g.t.min()) // L)
    nz = win[win > 0]
    t0 = time.perf_counter()
    exact = tm.count_exact(G, M, delta)
    t_exact = time.perf_counter() - t0
    log("exact", exact, f"{t_exact:.2f}s")
    t0 = time.perf_counter()
    tile, bpc = tm.batch_config(G, M, delta, c, p)
    t_tune = time.perf_counter() - t0
    log("autotuned tile", tile, "work-groups/CU", bpc, f"{t_tune:.2f}s")
    seeds = np.arange(64, dtype=np.uint64)

    def cold(sd):
        tm.batch_release(G)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = tm.estimate_batch(G, M, delta, c, p, sd)
        return time.perf_counter() - t0, out

    for w in range(args.warmup):
        dt_w, _ = cold(seeds + 500 * (w + 1))
        log("warmup", w, f"{dt_w:.2f}s")
    tm.profile_reset()
    tm.profile_enable(True)
    ts = []
    for i in range(args.steps):
        dt_i, _ = cold(seeds + 1000 * (i + 1))
        ts.append(dt_i)
        log("cold batch step", i, f"{dt_i:.2f}s")
    tm.profile_enable(False)
    t_vals = tm.profile_read("batch_anchor_values")
    warm = []
    for i in range(2):
        t0 = time.perf_counter()
        tm.estimate_batch(G, M, delta, c, p, seeds + 3000 + 100 * i)
        warm.append(time.perf_counter() - t0)
    log("warm replays", [f"{x:.2f}s" for x in warm])
    est, kept = tm.estimate_batch(G, M, delta, c, p, seeds)
    one = []
    t0 = time.perf_counter()
    for k, sd in enumerate(seeds):
        one.append(tm.estimate(G, M, delta, c, p, int(sd)))
        if k % 16 == 15:
            log("one at a time", k + 1, f"{time.perf_counter() - t0:.1f}s")
    t_seq = time.perf_counter() - t0
    assert all(a == b for a, b in zip(one, est)), "batched estimates differ from single calls"
    dt = float(np.mean(ts))
    mean, var = float(np.mean(est)), float(np.var(est, ddof=1))
    G.free()
    # the same comparison where one estimate is far from filling the GPU
    gs = ti.config_small_dense()
    Gs = tm.load_graph(gs.src, gs.dst, gs.t, gs.n)
    tm.estimate_batch(Gs, M, delta, c, p, seeds, tile=64)
    t0 = time.perf_counter()
    tm.estimate_batch(Gs, M, delta, c, p, seeds + 7, tile=64)
    small_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    for sd in seeds + 7:
        tm.estimate(Gs, M, delta, c, p, int(sd))
    small_seq = time.perf_counter() - t0
    Gs.free()
    log("small graph: batched", f"{small_batch * 1e3:.2f} ms, one at a time {small_seq * 1e3:.2f} ms")
    return {
        "metric": "temporal edges/s per motif query (batched p=0.1 estimates, cold)", "value": g.m * 64 / dt,
        "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "500k nodes, 50M edges, Zipf(1.8), bursty times over [0,3e8) s (sigma 1.5, phi 0.95, "
                               "30% silent hours); triangle, delta 3600, c 30, p 0.1, 64 seeds per call; a step "
                               "releases the cached batch state first",
                   "m": g.m, "n": g.n},
        "window_edges": {"windows": int(win.size), "nonempty": int(nz.size), "min": int(nz.min()),
                         "p50": int(np.median(nz)), "p99": int(np.percentile(nz, 99)), "max": int(nz.max())},
        "autotune": {"tile": tile, "workgroups_per_cu": bpc, "seconds": t_tune},
        "exact": {"count": exact, "seconds": t_exact},
        "estimates": {"mean": mean, "variance": var, "std_error": (var / 64) ** 0.5,
                      "rel_error_of_mean": (mean - exact) / exact if exact else None},
        "anchor_values_ms_per_step": t_vals[0] / max(1, args.steps),
        "warm_replay_s": warm, "one_at_a_time_s": t_seq, "cold_batch_s": dt, "batch_speedup_cold": t_seq / dt,
        "batch_speedup_warm": t_seq / float(np.mean(warm)),
        "small_graph_64_seeds": {"workload": "50 nodes, 20k uniform edges, triangle, delta 3600, c 30, p 0.1",
                                 "batched_ms": small_batch * 1e3, "one_at_a_time_ms": small_seq * 1e3,
                                 "speedup": small_seq / small_batch},
    }


def serving_queries(rng, sizes, n, qps):
    """Poisson arrivals at rate qps over graphs of the given edge counts;
    graph uniform; 25% exact / 75% estimate; motif uniform over the 36
    three-edge motifs and the 4-cycle; delta in {600, 3600, 86400}; p in
    {0.01, 0.1, 1}; c 30; a fresh 62-bit seed per request.  The 4-cycle (with
    delta at most 3600) and delta 86400 are drawn only on graphs of at most
    4e4 edges: on the larger graphs those queries cost seconds to minutes
    each."""
    motifs = THREE + [ti.CYCLE4]
    qs, t = [], 0.0
    for _ in range(n):
        t += rng.exponential(1.0 / qps)
        gi = int(rng.integers(0, len(sizes)))
        small = sizes[gi] <= 40_000
        M = motifs[int(rng.integers(0, len(motifs) - (0 if small else 1)))]
        deltas = [600, 3600, 86400] if (small and M != ti.CYCLE4) else [600, 3600]
        delta = int(rng.choice(deltas))
        if rng.random() < 0.25:
            qs.append(dict(at=t, graph=gi, edges=M, delta=delta, kind=0))
        else:
            qs.append(dict(at=t, graph=gi, edges=M, delta=delta, kind=1, c=30, p=float(rng.choice([0.01, 0.1, 1.0])),
                           seed=int(rng.integers(0, 1 << 62))))
    return qs


def _pct(a, f):
    """The f-quantile of a sorted array by the nearest-rank rule."""
    return float(a[max(0, int(np.ceil(f * len(a))) - 1)]) if len(a) else float("nan")


def serve_once(tm, Gs, sizes, qs, slots, budget):
    """Submit qs at their arrival times to a server; returns its statistics
    and the results in submission order."""
    S = tm.Server(slots=slots, budget_bytes=budget)
    ids = [S.add_graph(G) for G in Gs]
    tickets, t0 = [], time.perf_counter()
    for qi, q in enumerate(qs):
        now = time.perf_counter() - t0
        if now < q["at"]:
            time.sleep(q["at"] - now)
        tickets.append(S.submit(ids[q["graph"]], q["edges"], q["delta"], q["kind"], q.get("c", 0),
                                q.get("p", 0.0), q.get("seed", 0)))
        if qi % 100 == 99:
            log("  submitted", qi + 1, f"{time.perf_counter() - t0:.1f}s")
    res = []
    for k, tk in enumerate(tickets):
        res.append(S.wait(tk))
        if k % 100 == 99:
            log("  collected", k + 1, f"{time.perf_counter() - t0:.1f}s")
    st = S.stats()
    S.close()
    lat = np.sort(np.array([r["latency_ms"] for r in res]))
    big = np.sort(np.array([r["latency_ms"] for r, q in zip(res, qs) if sizes[q["graph"]] >= 10_000_000]))
    return {"p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"], "wall_s": st["wall_s"],
            "edges_per_s": st["edges_per_s"], "batches": st["batches"], "queries": st["completed"],
            "rejected": st["rejected"], "peak_workspace_bytes": st["peak_bytes"],
            "measured_max_bytes": st["measured_max_bytes"], "over_charge": st["over_charge"],
            "max_batch": max(r["batch_size"] for r in res),
            "p50_ms_check": _pct(lat, 0.5), "p99_ms_check": _pct(lat, 0.99),
            "p99_ms_graphs_from_1e7": _pct(big, 0.99)}, res


# The paper's timings for the 2-node motif (0,1),(1,0),(0,1) at delta 86400
# (its perf23 table; 16-core Xeon, C++): datasets by temporal-edge count, with
# the EX23 exact counter and EX23 with parallel sampling, in seconds.
PERF23_PAPER = {
    "CollegeMsg": (59_835, 0.017, 0.009),
    "SuperUser": (1_108_739, 1.097, 0.104),
    "WikiTalk": (6_100_000, 4.737, 0.876),
    "StackOverflow": (47_902_325, 108.1, 17.81),
}


def run_perf23(args):
    """Synthetic analogue of the paper's perf23 table: bursty Zipf(1.8)
    graphs with the temporal-edge counts of four of its datasets, the 2-node
    motif (0,1),(1,0),(0,1) at delta 86400 counted exactly and estimated
    (c 3, p 0.3: about 116 windows of 3 delta, a third kept; relative error
    against the exact count per seed), median of three runs each.  The paper's EX23 seconds on the dataset of the same size are
    quoted beside (other data, other hardware: context only)."""
    import torch
    import paper_1810_00980_amd as tm
    motif, delta, c, p = ti.TWO_NODE_ALT, 86400, 3, 0.3
    rows = []
    for name, (m, ex23_s, ex23ps_s) in PERF23_PAPER.items():
        g = ti.zipf_graph(max(1000, m // 30), m, 1.8, 30_000_000, 23)
        s_, d_, t_ = (torch.from_numpy(a).cuda() for a in (g.src, g.dst, g.t))
        G = tm.load_graph(s_, d_, t_, g.n)
        tm.count_exact_multi(G, [motif], delta)
        tm.estimate_multi(G, [motif], delta, c, p, 0)
        te, tz, exact, ests = [], [], 0, []
        for rep in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            exact = tm.count_exact_multi(G, [motif], delta)[0]
            torch.cuda.synchronize()
            te.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            z = tm.estimate_multi(G, [motif], delta, c, p, rep)[0][0]
            torch.cuda.synchronize()
            tz.append(time.perf_counter() - t0)
            ests.append(z)
        G.free()
        ex, es = float(np.median(te)), float(np.median(tz))
        rows.append({"like": name, "m": g.m, "n": g.n, "exact_count": exact, "exact_s": ex,
                     "exact_edges_per_s": g.m / ex, "estimate_s": es, "estimate_edges_per_s": g.m / es,
                     "estimate_rel_errors": [(z - exact) / exact if exact else None for z in ests],
                     "paper_ex23_s": ex23_s, "paper_ex23_ps_s": ex23ps_s})
        log("perf23", name, g.m, f"exact {ex * 1e3:.2f} ms, estimate {es * 1e3:.2f} ms")
    big = rows[-1]
    return {
        "metric": "temporal edges/s, 2-node motif (0,1),(1,0),(0,1), delta 86400 (exact count)",
        "value": big["exact_edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": 3, "warmup": 1,
        "ms_per_step": big["exact_s"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "bursty Zipf(1.8) graphs with the edge counts of four of the paper's datasets "
                               "(times over [0,3e7) s, n = m/30); the paper's perf23 workload shape; "
                               "estimates at c 3, p 0.3"},
        "sizes": rows,
    }


# The paper's timings for the bi-fan at delta 3600 (its bifan table; 16-core
# Xeon, C++ backtracking): datasets by temporal-edge count, exact and with
# parallel sampling, in seconds.
BIFAN_PAPER = {
    "CollegeMsg": (59_835, 0.081, 0.069),
    "Email-Eu": (332_334, 0.353, 0.120),
    "MathOverflow": (390_441, 0.528, 0.041),
    "AskUbuntu": (726_639, 1.408, 0.078),
    "SuperUser": (1_108_739, 2.486, 0.164),
}


def run_bifan(args):
    """Synthetic analogue of the paper's bifan table: the bi-fan
    (0,1),(0,2),(3,1),(3,2) at delta 3600 on bursty Zipf(1.8) graphs with the
    temporal-edge counts of its five datasets, counted exactly and estimated
    (c 30, p 0.1), one timed run each after a warm-up on the smallest.  The
    paper's backtracking seconds on the dataset of the same size are quoted
    beside (other data, other hardware: context only)."""
    import torch
    import paper_1810_00980_amd as tm
    delta, c, p = 3600, 30, 0.1
    rows = []
    for idx, (name, (m, bt_s, btps_s)) in enumerate(BIFAN_PAPER.items()):
        g = ti.zipf_graph(max(1000, m // 30), m, 1.8, 30_000_000, 23)
        s_, d_, t_ = (torch.from_numpy(a).cuda() for a in (g.src, g.dst, g.t))
        G = tm.load_graph(s_, d_, t_, g.n)
        if idx == 0:
            tm.count_exact(G, ti.BIFAN, delta)
            tm.estimate(G, ti.BIFAN, delta, c, p, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        exact = tm.count_exact(G, ti.BIFAN, delta)
        torch.cuda.synchronize()
        ex = time.perf_counter() - t0
        t0 = time.perf_counter()
        z = tm.estimate(G, ti.BIFAN, delta, c, p, 1)
        torch.cuda.synchronize()
        es = time.perf_counter() - t0
        G.free()
        rows.append({"like": name, "m": g.m, "n": g.n, "exact_count": exact, "exact_s": ex,
                     "exact_edges_per_s": g.m / ex, "estimate_s": es, "estimate_edges_per_s": g.m / es,
                     "estimate_rel_error": (z - exact) / exact if exact else None,
                     "paper_bt_s": bt_s, "paper_bt_ps_s": btps_s})
        log("bifan", name, g.m, f"exact {ex * 1e3:.1f} ms, estimate {es * 1e3:.1f} ms")
    big = rows[-1]
    return {
        "metric": "temporal edges/s, bi-fan (0,1),(0,2),(3,1),(3,2), delta 3600 (exact count)",
        "value": big["exact_edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": big["exact_s"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "bursty Zipf(1.8) graphs with the edge counts of the paper's five bi-fan datasets "
                               "(times over [0,3e7) s, n = m/30); estimates at c 30, p 0.1"},
        "sizes": rows,
    }


def run_four_edge(args):
    """The four-edge workload: 20M nodes, 500M edges, Zipf(2.0) endpoints,
    bursty times over [0, 3e8) s, drawn on the device, with the 4-star
    (0,1),(0,1),(0,2),(0,3) (its own counter) and the 4-cycle
    (0,1),(1,2),(2,3),(3,0) (the generic backtracking counter) at delta
    86400, c 30, p 0.05.  At full size the graph is generated and loaded
    (load time, device bytes) but not counted: one kept 30-day window holds
    about 2e12 star window-entry visits and the cycle about 1e17 three-edge
    prefixes, beyond a benchmark run.  Both motifs are timed, estimate and
    exact count, on the same recipe with 1% of the edges over the same span
    (200k nodes, 5M edges), whose hubs carry 1% of the density."""
    import torch
    import paper_1810_00980_amd as tm
    delta, c, p = 86400, 30, 0.05
    out = {"metric": "temporal edges/s per motif query (4-star and 4-cycle, exact and p=0.05 estimate)",
           "unit": "edges/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int64", "data": "synthetic"}
    sc = args.scale
    n, m_want, t_hi = int(20_000_000 * sc), int(500_000_000 * sc), int(300_000_000 * sc)
    t0 = time.perf_counter()
    if sc == 1.0:
        src, dst, t = ti.config_star_cycle()
    else:  # the same recipe and density on a fraction of the span
        src, dst, t = ti.zipf_graph_device(n, m_want, 2.0, t_hi, 3)
    torch.cuda.synchronize()
    m = int(src.numel())
    log("generated", m, "edges", f"{time.perf_counter() - t0:.1f}s")
    loads = []
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G = tm.load_graph(src, dst, t, n, exact_tables=False)
        torch.cuda.synchronize()
        loads.append(time.perf_counter() - t0)
        dev_bytes = G.device_bytes
        G.free()
        log("loaded", f"{loads[-1]:.2f}s", "device GB", dev_bytes / 1e9)
    del src, dst, t
    torch.cuda.empty_cache()
    full = {"workload": f"{n / 1e6:g}M nodes, {m / 1e6:g}M edges, Zipf(2.0) endpoints, bursty times over "
                        f"[0,{t_hi:.0e}) s (drawn on the device)", "m": m, "n": n, "scale": sc,
            "load_s": loads[-1], "load_edges_per_s": m / loads[-1], "graph_device_bytes": dev_bytes,
            "counted": False}
    # both motifs on the same recipe with 1% of the edges over the same span
    mv, nv = 5_000_000, 200_000
    src, dst, t = ti.zipf_graph_device(nv, mv, 2.0, 300_000_000, 5)
    Gs = tm.load_graph(src, dst, t, nv)
    del src, dst, t
    small = {"workload": "200k nodes, 5M edges, Zipf(2.0), bursty times over [0,3e8) s (graph seed 5)",
             "delta": delta, "c": c, "p": p}
    rates = []
    for M, name in ((ti.STAR4, "star4"), (ti.CYCLE4, "cycle4")):
        tm.estimate(Gs, M, delta, c, p, 0)
        ests = []
        for seed in range(1, 1 + args.steps):
            t0 = time.perf_counter()
            z = tm.estimate(Gs, M, delta, c, p, seed)
            ests.append({"seed": seed, "estimate": z, "s": time.perf_counter() - t0})
        dz = float(np.mean([e["s"] for e in ests]))
        t0 = time.perf_counter()
        ex = tm.count_exact(Gs, M, delta)
        de = time.perf_counter() - t0
        mean = float(np.mean([e["estimate"] for e in ests]))
        small[name] = {"estimates": ests, "estimate_s": dz, "exact": str(ex), "exact_s": de,
                       "estimate_edges_per_s": mv / dz, "exact_edges_per_s": mv / de,
                       "mean_estimate_rel_error": (mean - ex) / ex if ex else None}
        rates += [mv / dz, mv / de]
        log(name, "1% variant", f"estimate {dz:.2f}s exact {de:.2f}s", ex)
    Gs.free()
    q = 4
    wall = sum(small[k]["estimate_s"] + small[k]["exact_s"] for k in ("star4", "cycle4"))
    out.update({"value": mv * q / wall, "steps": args.steps, "warmup": 1, "ms_per_step": wall * 1e3,
                "config": {"workload": small["workload"] + "; the 1%-of-edges variant of the 500M-edge "
                                                           "four-edge workload; 4-star and 4-cycle, exact and "
                                                           "estimate, delta 86400, c 30, p 0.05",
                           "m": mv, "n": nv, "motif_queries_per_step": q},
                "full_size": full, "one_percent_variant": small})
    return out


def run_serve(args):
    """Poisson streams of count/estimate queries over the 8 resident graphs of
    1e4 .. 1e8 edges (or the first --serve-graphs of them) at several arrival
    rates, served by the
    continuous-batching server (4 slots, a device-memory budget on the
    workspace it measures) and, for comparison, one query at a time on the
    GPU in arrival order.  The value is the server's throughput at the
    highest rate whose p99 latency meets the stated target.  --serve-phase
    runs one side only (a line per phase, each with its per-query results);
    --serve-merge joins such lines into the comparison."""
    import torch
    import paper_1810_00980_amd as tm
    Gs, sizes = [], []
    for i in range(args.serve_graphs):
        s_, d_, t_, n = ti.serving_graph_device(i)
        Gs.append(tm.load_graph(s_, d_, t_, n))
        sizes.append(int(s_.numel()))
        del s_, d_, t_
    torch.cuda.empty_cache()
    log("graphs", sizes, "device GB", sum(G.device_bytes for G in Gs) / 1e9)
    slots, budget = 4, args.serve_budget_gib << 30

    def direct(q):
        G = Gs[q["graph"]]
        if q["kind"] == 0:
            return tm.count_exact(G, q["edges"], q["delta"])
        r = tm.estimate(G, q["edges"], q["delta"], q["c"], q["p"], q["seed"], info=(q["edges"] == ti.CYCLE4))
        return r["Z"] if isinstance(r, dict) else r

    warm = serving_queries(np.random.default_rng(1), sizes, 60, 1000.0)
    for q in warm:
        direct(q)
    serve_once(tm, Gs, sizes, warm, slots, budget)
    torch.cuda.synchronize()
    log("warm")
    phases = []
    for qps in args.qps_list:
        qs = serving_queries(np.random.default_rng(2024), sizes, args.queries, qps)
        edges = sum(sizes[q["graph"]] for q in qs)
        if args.serve_phase in ("both", "server"):
            log("qps", qps, "server")
            srv, res = serve_once(tm, Gs, sizes, qs, slots, budget)
            srv["results"] = [str(r["count"]) if q["kind"] == 0 else r["estimate"] for q, r in zip(qs, res)]
            srv["latency_ms"] = [round(r["latency_ms"], 3) for r in res]
            srv["batch_size"] = [r["batch_size"] for r in res]
            srv["graph_edges"] = [sizes[q["graph"]] for q in qs]
            phases.append({"qps": qps, "phase": "server", "queries": len(qs), "edges": edges, **srv})
            log("qps", qps, "server edges/s", f"{srv['edges_per_s']:.3e}", "p50", f"{srv['p50_ms']:.1f}", "p99",
                f"{srv['p99_ms']:.1f}")
        if args.serve_phase in ("both", "direct"):
            log("qps", qps, "one at a time")
            lat, got, t0 = [], [], time.perf_counter()
            for qi, q in enumerate(qs):
                now = time.perf_counter() - t0
                if now < q["at"]:
                    time.sleep(q["at"] - now)
                r = direct(q)
                lat.append(time.perf_counter() - t0 - q["at"])
                got.append(str(r) if q["kind"] == 0 else r)
                if qi % 100 == 99:
                    log("  done", qi + 1, f"{time.perf_counter() - t0:.1f}s")
            wall = time.perf_counter() - t0
            lat_ms = np.sort(np.array(lat) * 1e3)
            one = {"p50_ms": _pct(lat_ms, 0.5), "p99_ms": _pct(lat_ms, 0.99), "wall_s": wall,
                   "edges_per_s": edges / wall, "results": got, "latency_ms": [round(x * 1e3, 3) for x in lat],
                   "graph_edges": [sizes[q["graph"]] for q in qs]}
            phases.append({"qps": qps, "phase": "one_at_a_time", "queries": len(qs), "edges": edges, **one})
            log("qps", qps, "one at a time edges/s", f"{one['edges_per_s']:.3e}", "p50", f"{one['p50_ms']:.1f}",
                "p99", f"{one['p99_ms']:.1f}")
    for G in Gs:
        G.free()
    cfg = {"workload": f"{args.queries} Poisson queries per arrival rate over the {args.serve_graphs} graphs of "
                       f"1e4..{sizes[-1]:.2g} edges of the serving mix "
                       "(log-spaced, 100 edges per node, Zipf 1.8 endpoints, bursty times over "
                       "[0, max(1e6, 3m)) s); 25% exact / 75% estimate; motif uniform over 36 three-edge "
                       "motifs + 4-cycle (4-cycle, with delta <= 3600, and delta 86400 on graphs up to 4e4 "
                       "edges); delta in {600,3600,86400}; p in {0.01,0.1,1}; c 30; a fresh seed per "
                       "request", "graph_edges": sizes, "slots": slots, "budget_bytes": budget,
           "p99_target_ms": args.p99_target_ms}
    return serve_merge(phases, cfg, args.p99_target_ms)


def serve_merge(phases, cfg, target_ms):
    """One bench line from serving phases (the server and the one-at-a-time
    runs of each arrival rate, possibly from separate runs): per rate the two
    sides' latency and throughput, whether each meets the p99 target, and
    how many results differ between them (counts exactly, estimates beyond
    1e-12 relative)."""
    by = {}
    for ph in phases:
        by.setdefault(ph["qps"], {})[ph["phase"]] = ph
    sweeps = []
    for qps in sorted(by):
        d = by[qps]
        srv, one = d.get("server"), d.get("one_at_a_time")
        sw = {"qps": qps}
        for name, ph in (("server", srv), ("one_at_a_time", one)):
            if ph:
                sw[name] = {k: v for k, v in ph.items() if k not in ("results", "latency_ms", "batch_size", "qps",
                                                                      "phase", "graph_edges")}
                sw[name + "_meets_p99_target"] = ph["p99_ms"] <= target_ms
                if ph.get("latency_ms") and ph.get("graph_edges"):
                    # queries on the graphs below an eighth of the largest one's
                    # edges (the ones that need not wait for the large graphs)
                    big = max(ph["graph_edges"])
                    small = np.sort([l for l, e in zip(ph["latency_ms"], ph["graph_edges"]) if 8 * e < big])
                    large = np.sort([l for l, e in zip(ph["latency_ms"], ph["graph_edges"]) if 8 * e >= big])
                    sw[name]["small_graphs"] = {"queries": len(small), "p50_ms": _pct(small, 0.5),
                                                "p99_ms": _pct(small, 0.99)}
                    sw[name]["large_graphs"] = {"queries": len(large), "p50_ms": _pct(large, 0.5),
                                                "p99_ms": _pct(large, 0.99)}
        if srv and one:
            diff = 0
            for a, b in zip(srv["results"], one["results"]):
                if isinstance(a, str) or isinstance(b, str):
                    diff += int(str(a) != str(b))
                else:
                    diff += int(abs(a - b) > 1e-12 * abs(b))
            sw["results_differing_from_one_at_a_time"] = diff
            sw["server_over_one_at_a_time_throughput"] = srv["edges_per_s"] / one["edges_per_s"]
        sweeps.append(sw)
    ok = [sw for sw in sweeps if sw.get("server_meets_p99_target")]
    top = max(ok, key=lambda sw: sw["qps"]) if ok else next((sw for sw in sweeps if "server" in sw), None)
    cfg = dict(cfg, qps=sorted(by), value_at_qps=top["qps"] if top else None)
    return {"metric": "temporal edges/s per motif query (served stream); p50/p99 latency",
            "value": top["server"]["edges_per_s"] if top else None, "unit": "edges/s", "n_gpus": 1, "steps": 1,
            "warmup": 1, "ms_per_step": top["server"]["wall_s"] * 1e3 if top else None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic", "config": cfg,
            "sweep": sweeps, "phases": phases}


def _code_only(src: str) -> str:
    """C++ source without comments and blank space, so that a traffic record
    stays tied to the code it measured, not to how that code is annotated."""
    out, i, n = [], 0, len(src)
    while i < n:
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif src[i] in "\"'":
            q, j = src[i], i + 1
            while j < n and src[j] != q:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(src[i])
            i += 1
    return " ".join("".join(out).split())


def kernel_src_sha():
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(_code_only(open(f, encoding="utf-8").read()).encode())
    return h.hexdigest()


def traffic_file(kernel):
    return os.path.join(ROOT, "profiles", f"{kernel}_zipf10m_traffic.json")


def traffic_record(kernel):
    """HBM traffic of a sweep kernel from its committed rocprofv3 --pmc
    summary, valid only while the kernel source is unchanged."""
    if not os.path.exists(traffic_file(kernel)):
        return None
    rec = json.load(open(traffic_file(kernel)))
    sha = kernel_src_sha()
    if rec.get("kernel_src_sha256") != sha:
        return None
    return rec.get("traffic_bytes_per_launch")


# Algorithmic bytes per unit of the sweeps, the method's own work in the
# plain model (every anchor reads its edge: 16 B; every list entry in (t1, hi]
# it scans: 12 B, time and endpoint word; a weighted sweep also reads the
# entry's duration weight: 8 B; every binary-search probe of a closing-pair
# lookup: 8 B, counted by the census as ceil(log2(n + 1)) per search of a
# pair timeline of n entries, plus one probe to find the pair on a change).
# The exact-count tables let the 2-node and star counts skip their scans;
# their algorithmic bytes are still the scans they replace.
# The weighted triangles over static triangles (tm_tri_static_census): per
# (triangle, kept window) unit, the window bounds of its three pair
# timelines (six searches, 8 B each); per driver entry, its 16 B pair entry
# and the two 16 B entries where its middle and inner ranges start; per
# (first, last) pair visited, the inner 16 B pair entry and its 8 B weight.
PER_UNIT = {
    "sweep3": "16 B per anchor, 12 B per scanned entry, 8 B per weight read, 8 B per binary-search probe",
    "tri_static_weight": "48 B per (static triangle, kept window) unit, 48 B per driver entry, "
                         "24 B per (first, last) edge pair visited",
}


def sweep_bytes(exact, ests):
    out = {
        "sweep3_fwd_count": 16 * exact["anchors"] + 12 * exact["fwd_entries"],
        "sweep3_bwd_count": 16 * exact["anchors"] + 12 * exact["bwd_entries"],
        "sweep3_tri_count": 16 * exact["tri_anchors"] + 12 * exact["tri_entries"] + 8 * exact["tri_probes"],
        "sweep3_fwd_weight": 0, "sweep3_bwd_weight": 0, "sweep3_tri_weight": 0,
    }
    static = [e.get("static") for e in ests]
    if static and all(s is not None for s in static):
        out["tri_static_weight"] = sum(48 * s["units"] + 48 * s["drivers"] + 24 * s["combos"] for s in static)
    for e in ests:
        out["sweep3_fwd_weight"] += 16 * e["anchors"] + 20 * e["fwd_entries"]
        out["sweep3_bwd_weight"] += 16 * e["anchors"] + 20 * e["bwd_entries"]
        out["sweep3_tri_weight"] += 16 * e["tri_anchors"] + 20 * e["tri_entries"] + 8 * e["tri_probes"]
    return out


def sweep_roofline(exact, ests, kern, crit, alone, steps, traffic_records=True):
    """Roofline entry of the dominant sweep kernel.  The kernels of one pass
    run concurrently on forked streams and share the CUs, so each one's
    duration in the timed steps spans most of the pass; the dominant kernel
    is the one with the most time per step when each kernel of a pass runs
    alone (alone: one untimed step with the library's serial timing mode).
    achieved = its HBM bytes per launch (FETCH_SIZE + WRITE_SIZE from the
    committed rocprofv3 record of the current kernel source, calibrated by a
    plain copy) / its average launch duration in the timed steps; the
    algorithmic figure (census x per-unit bytes) is reported beside it.  When
    the record is stale (kernel source changed since the counters were
    taken), or when the step is not the workload the records were taken on
    (traffic_records false), traffic is null and frac falls back to the
    algorithmic figure, with frac_basis saying so."""
    bps = sweep_bytes(exact, ests)  # algorithmic bytes per step
    timed = {k: v for k, v in kern.items() if k in bps and v[1] > 0}
    if not timed:
        return None
    per = {}
    for k, (ms, n) in timed.items():
        per[k] = {"launches_per_step": n / steps, "avg_launch_ms": ms / n,
                  "algorithmic_bytes_per_launch": bps[k] * steps / n,
                  "algorithmic_GBs": bps[k] * steps / (ms / 1e3) / 1e9}
        tr = traffic_record(k) if traffic_records else None
        if tr is not None:
            per[k]["traffic_bytes_per_launch"] = tr
            per[k]["hbm_GBs"] = tr / (ms / n / 1e3) / 1e9
    dom = max(timed, key=lambda k: (alone.get(k, (0.0, 0))[0], timed[k][0]))
    d = per[dom]
    traffic = d.get("traffic_bytes_per_launch")
    if traffic is not None:
        ach, basis = d["hbm_GBs"], "rocprofv3 FETCH_SIZE + WRITE_SIZE per launch / launch time"
    else:
        ach, basis = d["algorithmic_GBs"], ("algorithmic bytes per launch / launch time (counter record stale)"
                                            if traffic_records else
                                            "algorithmic bytes per launch / launch time (no counter record of "
                                            "this workload)")
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": traffic, "frac_basis": basis, "kernel": dom, "avg_launch_ms": d["avg_launch_ms"],
            "launches": timed[dom][1],
            "algorithmic": {"bytes_per_launch": d["algorithmic_bytes_per_launch"], "GBs": d["algorithmic_GBs"],
                            "frac": d["algorithmic_GBs"] / HBM_PEAK_GBS,
                            "per_unit": PER_UNIT.get(dom, PER_UNIT["sweep3"])},
            "census": {"exact": exact, "estimates": ests}, "sweep_kernels": per,
            "sweep_kernels_ms_per_step": {k: v[0] / steps for k, v in kern.items()},
            "critical_path_ms_per_step": {k: v[0] / steps for k, v in crit.items() if v[1] > 0},
            "alone_ms_per_step": {k: v[0] for k, v in alone.items() if v[1] > 0}}


# rocprofv3 names of the sweep kernels (template arguments: mode, forward,
# class mask) and the library's timing names
TEMPLATE_NAMES = {"k_sweep3<0, true, 7u>": "sweep3_fwd_count", "k_sweep3<0, true, 8u>": "sweep3_tri_count",
                  "k_sweep3<0, false, 0u>": "sweep3_bwd_count", "k_sweep3<1, true, 7u>": "sweep3_fwd_weight",
                  "k_sweep3<1, true, 8u>": "sweep3_tri_weight", "k_sweep3<1, false, 0u>": "sweep3_bwd_weight",
                  "k_st_weight<false>": "tri_static_weight"}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def _csv_rows(folder, suffix):
    rows = []
    for f in sorted(glob.glob(os.path.join(folder, "**", f"*{suffix}"), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {folder} (run rocprofv3 with -f csv)")
    return rows


def _short_name(kernel_name):
    """A rocprofv3 kernel name without return type, namespaces and arguments."""
    k = kernel_name.strip()
    if k.startswith("void "):
        k = k[5:]
    k = k.replace("(anonymous namespace)::", "").replace("sweepdev::", "")
    return k.split("(")[0].strip()


def _timing_name(kernel_name):
    return TEMPLATE_NAMES.get(_short_name(kernel_name))


def pmc_summary(fetch_dir, write_dir):
    """Per sweep kernel: mean FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
    over its dispatches, each scaled by what the counter reads for the 1 GiB
    copy of --copy-calib (1 GiB read, 1 GiB written), written with the
    kernel source hash to profiles/<kernel>_zipf10m_traffic.json."""
    vals = {}
    for folder, counter in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        per = {}
        copy = 0.0
        for r in _csv_rows(folder, "counter_collection.csv"):
            if r.get("Counter_Name") != counter:
                continue
            v = float(r["Counter_Value"])
            k = r["Kernel_Name"]
            if _short_name(k) == COPY_KERNEL:
                copy = max(copy, v)
            name = _timing_name(k)
            if name:
                per.setdefault(name, []).append(v)
        if copy <= 0:
            raise SystemExit(f"no {COPY_KERNEL} dispatch in {folder}: run bench.py with --copy-calib")
        vals[counter] = (per, copy)
    sha = kernel_src_sha()
    fper, fcopy = vals["FETCH_SIZE"]
    wper, wcopy = vals["WRITE_SIZE"]
    ff, wf = (1 << 20) / fcopy, (1 << 20) / wcopy  # KiB of 1 GiB over what each counter read
    for name in sorted(set(fper) & set(wper)):
        fk, wk = sum(fper[name]) / len(fper[name]), sum(wper[name]) / len(wper[name])
        rec = {"kernel": f"{[t for t, n in TEMPLATE_NAMES.items() if n == name][0]} ({name})",
               "workload": "zipf10m bench step (100k nodes, 10M edges, 36 three-edge motifs, delta 3600)",
               "kernel_src_sha256": sha,
               "commands": [f"rocprofv3 --pmc FETCH_SIZE -f csv -d REPO/{fetch_dir} -o run -- python3 REPO/bench.py "
                            "--profile-run --copy-calib",
                            f"rocprofv3 --pmc WRITE_SIZE -f csv -d REPO/{write_dir} -o run -- python3 REPO/bench.py "
                            "--profile-run --copy-calib",
                            f"python3 bench.py --pmc-summary {fetch_dir} {write_dir}"],
               "dispatches_averaged": len(fper[name]),
               "fetch_size_kib_per_dispatch": fk, "write_size_kib_per_dispatch": wk,
               "calibration": {"copy": "1 GiB device-to-device copy (1 GiB read + 1 GiB written)",
                               "copy_fetch_kib": fcopy, "copy_write_kib": wcopy,
                               "fetch_factor": ff, "write_factor": wf},
               "traffic_bytes_per_launch": (fk * ff + wk * wf) * 1024}
        with open(traffic_file(name), "w") as fh:
            json.dump(rec, fh, indent=1)
        print(name, f"{rec['traffic_bytes_per_launch'] / 1e9:.2f} GB per launch", file=sys.stderr)


PMC_COUNTERS = ("TCC_HIT_sum", "TCC_MISS_sum", "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_BUSY_CYCLES",
                "TA_BUSY_avr", "GRBM_GUI_ACTIVE")
N_XCD = 8  # MI355X: GRBM_GUI_ACTIVE sums one instance per XCD


def pmc_counters(folder):
    """Per sweep kernel: the mean over its dispatches of the counters of one
    rocprofv3 --pmc pass (PMC_COUNTERS), with the L2 hit rate (TCC hits over
    hits and misses), the shares of wave cycles spent waiting for anything
    (SQ_WAIT_ANY: memory and dependencies) and waiting to issue
    (SQ_WAIT_INST_ANY), both over SQ_WAVE_CYCLES (all in quad-cycles), and
    the texture-address units' busy share (TA_BUSY_avr, the mean over the
    units, over the busy cycles of one XCD: GRBM_GUI_ACTIVE / N_XCD),
    written to profiles/sweep3_zipf10m_counters.json."""
    per = {}
    for r in _csv_rows(folder, "counter_collection.csv"):
        name = _timing_name(r["Kernel_Name"])
        if not name or r.get("Counter_Name") not in PMC_COUNTERS:
            continue
        per.setdefault(name, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    out = {"workload": "zipf10m bench step (100k nodes, 10M edges, 36 three-edge motifs, delta 3600)",
           "kernel_src_sha256": kernel_src_sha(),
           "commands": [f"rocprofv3 --pmc {' '.join(PMC_COUNTERS)} -f csv -d REPO/{folder} -o run -- "
                        "python3 REPO/bench.py --profile-run",
                        f"python3 bench.py --pmc-counters {folder}"],
           "kernels": {}}
    for name, cs in sorted(per.items()):
        mean = {c: sum(v) / len(v) for c, v in cs.items()}
        rec = {"dispatches_averaged": max(len(v) for v in cs.values()), "mean_per_dispatch": mean}
        h, mi = mean.get("TCC_HIT_sum"), mean.get("TCC_MISS_sum")
        if h is not None and mi is not None and h + mi > 0:
            rec["l2_hit_rate"] = h / (h + mi)
        wc = mean.get("SQ_WAVE_CYCLES")
        for c, key in (("SQ_WAIT_ANY", "wave_cycles_waiting_share"),
                       ("SQ_WAIT_INST_ANY", "wave_cycles_waiting_issue_share")):
            if mean.get(c) is not None and wc:
                rec[key] = mean[c] / wc
        ta, g = mean.get("TA_BUSY_avr"), mean.get("GRBM_GUI_ACTIVE")
        if ta is not None and g:
            rec["ta_busy_share"] = ta / (g / N_XCD)
        out["kernels"][name] = rec
        print(name, {k: round(v, 3) for k, v in rec.items() if isinstance(v, float)}, file=sys.stderr)
    with open(os.path.join(ROOT, "profiles", "sweep3_zipf10m_counters.json"), "w") as fh:
        json.dump(out, fh, indent=1)


def kt_summary(folder):
    """Kernel-trace summary of a --profile-run: per kernel, calls, total and
    average duration; for the sweep kernels only the timed step's dispatches
    (the second half of each one's dispatches: the serial-timing step runs
    the same launches first)."""
    rows = _csv_rows(folder, "kernel_trace.csv")
    per = {}
    for r in rows:
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        name = _short_name(r["Kernel_Name"])
        per.setdefault(name, []).append(dur)
    for name in list(per):
        if name in TEMPLATE_NAMES:
            d = per[name]
            per[name] = d[len(d) // 2:]
    tot = sum(sum(v) for v in per.values())
    lines = ["rocprofv3 kernel trace: one timed bench step on the 10M-edge Zipf(1.8) workload", "",
             "commands (REPO = repository root; run from /tmp with TMPDIR=/tmp):",
             f"  rocprofv3 --kernel-trace --stats -f csv -d REPO/{folder} -o run -- python3 REPO/bench.py --profile-run",
             f"  python3 bench.py --kt-summary {folder}", "",
             "workload: 100k nodes, 10M edges, Zipf(1.8) endpoints, bursty times over [0,3e7) s, 36 three-edge "
             "motifs, delta 3600;", "one step = load + exact counts + estimates at c in {10,30} x p in {0.01,0.1}; "
             "durations in microseconds;", "sweep kernels: the timed step's dispatches only (they run "
             "concurrently on forked streams, so each spans most of its pass)", "",
             f"{'kernel':<60} {'calls':>7} {'total_us':>14} {'avg_us':>14} {'pct':>7}"]
    for name, d in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:40]:
        label = name + (f" ({TEMPLATE_NAMES[name]})" if name in TEMPLATE_NAMES else "")
        lines.append(f"{label[:60]:<60} {len(d):>7} {sum(d):>14.1f} {sum(d) / len(d):>14.1f} "
                     f"{100 * sum(d) / tot:>7.2f}")
    out = os.path.join(ROOT, "profiles", "sweep3_zipf10m_kernel_trace.txt")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines[-12:]), file=sys.stderr)


def latency(fn, repeats):
    """p50 / p99 (nearest rank) and mean of `repeats` timed calls, in ms."""
    import torch
    ts = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        ts.append((time.perf_counter() - t0) * 1e3)
    ts.sort()
    pct = lambda f: ts[max(0, int(np.ceil(f * len(ts))) - 1)]
    return {"repeats": repeats, "p50_ms": pct(0.5), "p99_ms": pct(0.99), "mean_ms": float(np.mean(ts))}


def stream_estimates(tm, torch, g, motifs, delta, c=30, p=0.1):
    """The p = 0.1 estimates of all the step's motifs from the time-sorted
    edges in host memory, one kept window on the device at a time: time per
    call (uploads included), the largest resident window and its graph's
    device bytes, beside the in-memory graph's; results are checked equal to
    the in-memory call."""
    o = np.argsort(g.t, kind="stable")
    hs, hd, ht = g.src[o], g.dst[o], g.t[o]
    tm.estimate_stream(hs, hd, ht, g.n, motifs, delta, c, p, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est, _, info = tm.estimate_stream(hs, hd, ht, g.n, motifs, delta, c, p, 0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s_, d_, t_ = (torch.from_numpy(a).cuda() for a in (g.src, g.dst, g.t))
    G = tm.load_graph(s_, d_, t_, g.n)
    same = est == tm.estimate_multi(G, motifs, delta, c, p, 0)[0]
    full = G.device_bytes
    G.free()
    return {"c": c, "p": p, "ms": dt * 1e3, "edges_per_s_per_query": g.m * len(motifs) / dt,
            "kept_windows": info["n_kept"], "max_window_edges": info["max_window_edges"],
            "peak_window_graph_bytes": info["peak_graph_bytes"], "in_memory_graph_bytes": full,
            "same_results": same}


def edge_proportional(tm, torch, g, src, dst, t, motifs, delta, c=30):
    """Algorithm 1 with the paper's window probabilities q_j = min(1, r |T_j| / |T|)
    (equation heuristic_q) and b shifts, for all the step's motifs: r = 0.1 J
    keeps about as many windows as p = 0.1.  Also the paper's diagnostic of
    how well q follows the weighted counts: with every window of one shift
    kept, the correlation of each window's edge count with the triangle's
    weighted count Y_{s,j}."""
    G = tm.load_graph(src, dst, t, g.n)
    L = c * delta
    tn = np.sort(g.t - g.t.min())
    J = 1 + -(-int(tn[-1]) // L)
    r = 0.1 * J
    out = {"c": c, "r": r, "windows": J}
    for b in (1, 4):
        tm.estimate_q(G, motifs, delta, c, r, b, 0, cap=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, w = tm.estimate_q(G, motifs, delta, c, r, b, 1, cap=0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"b{b}"] = {"ms": dt * 1e3, "edges_per_s_per_query": g.m * len(motifs) / dt, "kept_windows": w["n_kept"]}
    s0 = tm.estimate(G, ti.TRIANGLE, delta, c, 1e-300, 0, info=True)["s"]
    _, w = tm.estimate_q(G, [ti.TRIANGLE], delta, c, 1e15, 1, 0, cap=J + 1)
    lo = s0 + (w["j"] - 1) * L
    cnt = np.searchsorted(tn, lo + L - 1, side="right") - np.searchsorted(tn, lo, side="left")
    out["all_windows_kept"] = int(w["n_kept"])
    out["corr_window_edges_vs_triangle_Y"] = float(np.corrcoef(cnt, w["y"][:, 0])[0, 1])
    G.free()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="zipf10m",
                    choices=sorted(WORKLOADS) + ["batch50m", "serve", "perf23", "bifan", "zipf500m_star_cycle"])
    ap.add_argument("--scale", type=float, default=1.0,
                    help="zipf500m_star_cycle: fraction of the nodes, edges and time span of the loaded graph "
                         "(same density)")
    ap.add_argument("--qps-list", type=float, nargs="+", default=[2.0, 4.0, 8.0], help="serve: arrival rates")
    ap.add_argument("--queries", type=int, default=1000, help="serve: queries per arrival rate")
    ap.add_argument("--p99-target-ms", type=float, default=5000.0, help="serve: the stated p99 latency target")
    ap.add_argument("--serve-budget-gib", type=int, default=16, help="serve: the server's device-memory budget")
    ap.add_argument("--serve-graphs", type=int, default=8, choices=range(1, 9),
                    help="serve: the first K of the 8 graphs of 1e4..1e8 edges")
    ap.add_argument("--serve-phase", choices=["both", "server", "direct"], default="both",
                    help="serve: run the server, the one-at-a-time comparison, or both")
    ap.add_argument("--serve-merge", nargs="+", metavar="JSON",
                    help="join the serve lines of separate phase runs into one line and exit")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the serial-timing step and one timed step (for rocprofv3 runs)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic records from two rocprofv3 --pmc -f csv runs and exit")
    ap.add_argument("--kt-summary", metavar="DIR", help="write the kernel-trace summary of a --profile-run and exit")
    ap.add_argument("--pmc-counters", metavar="DIR",
                    help="write the L2, wait and TA counter summary of a rocprofv3 --pmc pass and exit")
    ap.add_argument("--latency-repeats", type=int, default=50)
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.kt_summary:
        kt_summary(args.kt_summary)
        return
    if args.pmc_counters:
        pmc_counters(args.pmc_counters)
        return
    if args.serve_merge:
        lines = [json.loads(open(f).read().strip().splitlines()[-1]) for f in args.serve_merge]
        print(json.dumps(serve_merge([ph for ln in lines for ph in ln["phases"]], lines[0]["config"],
                                     lines[0]["config"]["p99_target_ms"])))
        return
    if args.profile_run:
        args.steps, args.warmup, args.no_cpu = 1, 0, True
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the multi-GPU sharding of "
              "windows is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("RANK", "0")) != 0:
        return

    import torch
    import paper_1810_00980_amd as tm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload in ("batch50m", "serve", "perf23", "bifan", "zipf500m_star_cycle"):
        out = {"batch50m": run_batch, "serve": run_serve, "perf23": run_perf23, "bifan": run_bifan,
               "zipf500m_star_cycle": run_four_edge}[args.workload](args)
        print(json.dumps(out), flush=True)
        return
    W = WORKLOADS[args.workload]
    motifs, delta = W["motifs"], W["delta"]
    log("generating", args.workload)
    g = W["graph"]()
    src, dst, t = (torch.from_numpy(a).cuda() for a in (g.src, g.dst, g.t))
    torch.cuda.synchronize()

    if args.copy_calib:
        x = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")

    def step(times):
        t0 = time.perf_counter()
        G = tm.load_graph(src, dst, t, g.n)
        t1 = time.perf_counter()
        exact = tm.count_exact_multi(G, motifs, delta)
        t2 = time.perf_counter()
        ests = []
        for (c, p) in W["est"]:
            z, _ = tm.estimate_multi(G, motifs, delta, c, p, 0)
            ests.append(z)
        t3 = time.perf_counter()
        G.free()
        if times is not None:
            times["load"].append(t1 - t0)
            times["exact"].append(t2 - t1)
            times["est"].append(t3 - t2)
        return exact, ests

    for i in range(args.warmup):
        step(None)
        log("warmup", i)
    # one untimed step with each pass's kernels run one after another, which
    # gives every kernel's own duration (this decides the dominant kernel)
    tm.profile_reset()
    tm.profile_enable(True, serial=True)
    step(None)
    torch.cuda.synchronize()
    tm.profile_enable(False)
    alone = {k: tm.profile_read(k) for k in SWEEP_KERNELS}
    log("serial step done")
    tm.profile_reset()
    tm.profile_enable(True)
    times = {"load": [], "exact": [], "est": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        exact, ests = step(times)
        log("step", i, f"{time.perf_counter() - t0:.2f}s")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    tm.profile_enable(False)
    kern = {k: tm.profile_read(k) for k in SWEEP_KERNELS}
    crit = {k: tm.profile_read("crit:" + k) for k in SWEEP_KERNELS}
    if args.profile_run:
        log("profile run done", {k: v for k, v in kern.items()})
        return

    # The same step with its queries issued together from one host thread
    # each, on streams of their own (the library keeps per-thread workspaces
    # and side streams), so that short passes fill the tails of long ones.
    # Reported beside the sequential figure, which stays `value` because the
    # roofline is read from the sequential steps' kernel durations.
    streams = [torch.cuda.Stream() for _ in range(1 + len(W["est"]))]

    def step_concurrent():
        G = tm.load_graph(src, dst, t, g.n)
        out = [None] * len(streams)

        def run(k):
            if k == 0:
                out[0] = tm.count_exact_multi(G, motifs, delta, stream=streams[0])
            else:
                c, p = W["est"][k - 1]
                out[k] = tm.estimate_multi(G, motifs, delta, c, p, 0, stream=streams[k])[0]
        threads = [threading.Thread(target=run, args=(k,)) for k in range(len(streams))]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        G.free()
        return out

    same = step_concurrent() == [exact] + ests
    torch.cuda.synchronize()
    tc0 = time.perf_counter()
    for i in range(args.steps):
        step_concurrent()
    torch.cuda.synchronize()
    dtc = (time.perf_counter() - tc0) / args.steps
    log("concurrent steps done", f"{dtc * 1e3:.1f} ms per step")
    edge_prop = edge_proportional(tm, torch, g, src, dst, t, motifs, delta)
    log("edge-proportional estimates done")
    streaming = stream_estimates(tm, torch, g, motifs, delta)
    log("streaming estimates done")

    q = len(motifs) * (1 + len(W["est"]))
    G = tm.load_graph(src, dst, t, g.n)
    census = tm.sweep_census(G, delta)
    ests = [tm.sweep_census_est(G, delta, c, p, 0) for c, p in W["est"]]
    for e, (c, p) in zip(ests, W["est"]):
        try:
            e["static"] = tm.tri_static_census(G, delta, c, p, 0)
        except tm.TMError:
            e["static"] = None  # no static triangles kept: the list sweep counts them
    tables = G.exact_table_bytes > 0
    # latency over repeated single queries on the resident graph: the exact
    # pass of every motif, the p = 0.1 estimate pass (largest c), and one
    # motif (the triangle) alone
    cl, pl = max(W["est"], key=lambda e: (e[1], e[0]))
    R = args.latency_repeats
    lat = {"exact_all_motifs": latency(lambda: tm.count_exact_multi(G, motifs, delta), R),
           f"estimate_all_motifs_c{cl}_p{pl}": latency(lambda: tm.estimate_multi(G, motifs, delta, cl, pl, 0), R),
           "exact_triangle": latency(lambda: tm.count_exact(G, ti.TRIANGLE, delta), R),
           f"estimate_triangle_c{cl}_p{pl}": latency(lambda: tm.estimate(G, ti.TRIANGLE, delta, cl, pl, 0), R)}
    for v in lat.values():
        v["edges_per_s_per_query_at_p50"] = None
    lat["exact_all_motifs"]["edges_per_s_per_query_at_p50"] = g.m * len(motifs) / (lat["exact_all_motifs"]["p50_ms"] / 1e3)
    k_est = f"estimate_all_motifs_c{cl}_p{pl}"
    lat[k_est]["edges_per_s_per_query_at_p50"] = g.m * len(motifs) / (lat[k_est]["p50_ms"] / 1e3)
    lat["exact_triangle"]["edges_per_s_per_query_at_p50"] = g.m / (lat["exact_triangle"]["p50_ms"] / 1e3)
    k_tri = f"estimate_triangle_c{cl}_p{pl}"
    lat[k_tri]["edges_per_s_per_query_at_p50"] = g.m / (lat[k_tri]["p50_ms"] / 1e3)
    log("latency repeats done")
    G.free()
    roofline = sweep_roofline(census, ests, kern, crit, alone, args.steps,
                              traffic_records=args.workload == "zipf10m")
    if roofline:
        roofline["exact_tables"] = tables
    out = {
        "metric": "temporal edges/s per motif query (exact & p=0.1 estimate) vs CPU",
        "value": g.m * q / dt, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": W["desc"], "m": g.m, "n": g.n, "motif_queries_per_step": q},
        "phases_ms": {k: 1e3 * float(np.mean(v)) for k, v in times.items()},
        "exact_edges_per_s_per_query": g.m * len(motifs) / float(np.mean(times["exact"])),
        "estimate_p0.1_edges_per_s_per_query": g.m * len(motifs) / (lat[k_est]["mean_ms"] / 1e3),
        "latency": lat,
        "roofline": roofline,
        "concurrent_queries": {"ms_per_step": dtc * 1e3, "value": g.m * len(motifs) * (1 + len(W["est"])) / dtc,
                               "threads": len(streams), "same_results": same},
        "edge_proportional": edge_prop,
        "streaming": streaming,
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(g, motifs, delta)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
