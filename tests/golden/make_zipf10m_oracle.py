"""Writes tests/golden/zipf10m_oracle.json: the oracle's values on the
10M-edge Zipf(1.8) workload (100k nodes, bursty times over [0, 3e7) s,
graph seed 2), all 36 three-edge motifs at delta 3600:

* exact whole-graph counts C_M (Sec. 2, Definition "motif delta-instance");
* Algorithm 1 (Sec. 4) with one shift and q_j = p at c in {10, 30} and
  p in {0.01, 0.1}, estimator seed 0: shift, number of windows, kept
  windows, per-motif kept-window counts and estimates Z.

Only the oracle (tier C, oracle.count3_indexed / oracle.estimate3_indexed)
and the seeded input generator are called.  Takes about an hour on 6 host
threads:  python tests/golden/make_zipf10m_oracle.py [threads]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import tm_inputs as ti  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zipf10m_oracle.json")
DELTA = 3600
SETTINGS = [(10, 0.01), (10, 0.1), (30, 0.01), (30, 0.1)]


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    g = ti.config_zipf10m()
    motifs = ti.three_edge_motifs()
    out = {"workload": "config_zipf10m(): 100k nodes, 10M edges, Zipf(1.8), bursty times over [0, 3e7) s, seed 2",
           "delta": DELTA, "motifs": [list(map(list, M)) for M in motifs], "estimates": []}
    t0 = time.time()
    for c, p in SETTINGS:
        r = oracle.estimate3_indexed(g.src, g.dst, g.t, motifs, DELTA, c, p, 0, threads=threads)
        out["estimates"].append({"c": c, "p": p, "seed": 0, "s": r["s"], "J": r["J"], "n_kept": r["n_kept"],
                                 "kept": [int(j) for j in r["kept"]],
                                 "kept_counts": [str(k) for k in r["kept_counts"]], "Z": r["Z"]})
        print(f"estimate c={c} p={p}: {r['n_kept']} kept windows, {time.time() - t0:.0f} s", flush=True)
    counts = oracle.count3_indexed(g.src, g.dst, g.t, motifs, DELTA, threads=threads)
    out["exact"] = [str(x) for x in counts]
    print(f"exact counts: {time.time() - t0:.0f} s", flush=True)
    out["oracle_seconds"] = time.time() - t0
    with open(OUT + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
