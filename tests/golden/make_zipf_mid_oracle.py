"""Writes tests/golden/zipf_mid_oracle.json: the oracle's values on a
300k-edge graph drawn with the recipe of the 10M-edge workload (Zipf(1.8)
endpoints, bursty hourly rates, one edge per 3 s on average, 100 edges per
node: 3,000 nodes, times over [0, 9e5) s, graph seed 12), all 36
three-edge motifs at delta 3600:

* exact whole-graph counts C_M (Sec. 2, Definition "motif delta-instance");
* Algorithm 1 (Sec. 4) with one shift and q_j = p at c in {10, 30},
  p in {0.01, 0.1}, estimator seeds 0..7: shift, kept windows, per-motif
  kept-window counts and estimates Z.

Only the oracle (tier C) and the seeded input generator are called:
python tests/golden/make_zipf_mid_oracle.py [threads]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import tm_inputs as ti  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zipf_mid_oracle.json")
DELTA = 3600


def graph():
    return ti.zipf_graph(3000, 300_000, 1.8, 900_000, 12)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    g = graph()
    motifs = ti.three_edge_motifs()
    out = {"workload": "zipf_graph(3000, 300000, 1.8, 900000, 12)", "delta": DELTA,
           "motifs": [list(map(list, M)) for M in motifs], "estimates": []}
    t0 = time.time()
    for c in (10, 30):
        for p in (0.01, 0.1):
            for seed in range(8):
                r = oracle.estimate3_indexed(g.src, g.dst, g.t, motifs, DELTA, c, p, seed, threads=threads)
                out["estimates"].append({"c": c, "p": p, "seed": seed, "s": r["s"], "J": r["J"],
                                         "n_kept": r["n_kept"], "kept": [int(j) for j in r["kept"]],
                                         "kept_counts": [str(k) for k in r["kept_counts"]], "Z": r["Z"]})
    out["exact"] = [str(x) for x in oracle.count3_indexed(g.src, g.dst, g.t, motifs, DELTA, threads=threads)]
    out["oracle_seconds"] = time.time() - t0
    print(f"{time.time() - t0:.0f} s", flush=True)
    with open(OUT + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
