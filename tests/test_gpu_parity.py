"""GPU parity: libtm (HIP, gfx950) against the CPU oracle on the same seeded
inputs.  Counts and histograms must be bit-exact; estimates for the same seed
within 1e-12 relative (the weighting is the same fixed-order FP64 sum, so in
practice they are identical)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import tm_inputs as ti

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_1810_00980_amd as tm
    return tm


def say(*a):
    print("[case]", *a, flush=True)


def to_dev(g):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (g.src, g.dst, g.t)]


def load(tm, g, device=True, exact_tables=True):
    if device:
        s, d, t = to_dev(g)
        return tm.load_graph(s, d, t, g.n, exact_tables=exact_tables)
    return tm.load_graph(g.src, g.dst, g.t, g.n, exact_tables=exact_tables)


def close(a, b):
    return abs(a - b) <= REL * max(1.0, abs(b))


MOTIFS = ti.three_edge_motifs() + [ti.CYCLE4, ti.STAR4, ti.OUTSTAR5, ti.BIFAN, ((0, 1),), ((0, 1), (1, 0)),
                                    ((0, 1), (2, 0)), ((0, 1), (0, 1)), ((0, 1), (1, 2), (2, 3)),
                                    ((0, 1), (1, 2), (2, 0), (0, 1)),
                                    # second edge from an in-list; a repeated pair at level 2
                                    ((0, 1), (2, 1), (1, 3), (3, 2)), ((0, 1), (1, 2), (0, 1), (2, 0))]
FOUR = [M for M in MOTIFS if len(M) == 4]


@pytest.mark.parametrize("seed", range(4))
def test_small_random_all_motifs(tm, seed):
    # dense tiny graphs: many repeated pairs, ties and self-loops; several
    # 256-anchor tiles and a ragged tail
    g = ti.random_small_graph(6 + seed, 700 + 37 * seed, 3000, 900 + seed, allow_self_loops=True)
    say("small_random", seed, g.m)
    G = load(tm, g, device=(seed % 2 == 0))
    nl = g.src != g.dst
    assert G.n_pairs == len(set(zip(g.src[nl].tolist(), g.dst[nl].tolist())))
    for M in MOTIFS:
        for delta in (0, 7, 60):
            got = tm.count_exact(G, M, delta)
            want, _ = oracle.count(g.src, g.dst, g.t, M, delta, hist=False)
            assert got == want, (M, delta, got, want)
    for ms in (MOTIFS[:8], FOUR):
        cnt, hlo, hhi = tm.count_exact_multi(G, ms, 60, hist=True)
        for i, M in enumerate(ms):
            want, h = oracle.count(g.src, g.dst, g.t, M, 60)
            assert cnt[i] == want and (hlo[i] == h).all() and not hhi[i].any(), M


@pytest.mark.parametrize("motif", [ti.TRIANGLE, ti.TWO_NODE_ALT, ((0, 1), (0, 2), (2, 0)), ti.CYCLE4])
def test_estimate_matches_oracle_seed_by_seed(tm, motif):
    g = ti.random_small_graph(7, 900, 5000, 31, allow_self_loops=True)
    say("estimate", motif)
    G = load(tm, g)
    for (delta, c, p) in ((40, 2, 0.5), (40, 3, 1.0), (25, 10, 0.2)):
        for seed in range(6):
            r = tm.estimate(G, motif, delta, c, p, seed, info=True)
            o = oracle.estimate(g.src, g.dst, g.t, motif, delta, c, p, seed)
            assert r["s"] == o["s"] and r["J"] == o["J"] and r["n_kept"] == o["n_kept"]
            assert list(r["kept"]) == list(o["kept"])
            assert list(r["win_counts"]) == list(o["win_counts"])
            assert (r["hist_lo"] == o["hist"]).all() and not r["hist_hi"].any()
            assert r["kept_count"] == int(o["win_counts"].sum())
            assert close(r["Z"], o["Z"]), (r["Z"], o["Z"])


def test_small_config_exact_and_estimate(tm):
    """1,000 nodes, 20,000 uniform edges, triangle, delta 3600, c 30, p 0.1,
    seed 0; and the 50-node version where the count is not zero."""
    for g in (ti.config_small(), ti.config_small_dense()):
        say("small_config", g.n)
        G = load(tm, g)
        delta, c, p = 3600, 30, 0.1
        want, h = oracle.count(g.src, g.dst, g.t, ti.TRIANGLE, delta)
        cnt, hlo, _ = tm.count_exact_multi(G, [ti.TRIANGLE], delta, hist=True)
        assert cnt[0] == want and (hlo[0] == h).all()
        for seed in (0, 1, 2):
            r = tm.estimate(G, ti.TRIANGLE, delta, c, p, seed, info=True)
            o = oracle.estimate(g.src, g.dst, g.t, ti.TRIANGLE, delta, c, p, seed)
            assert list(r["kept"]) == list(o["kept"]) and list(r["win_counts"]) == list(o["win_counts"])
            assert close(r["Z"], o["Z"])


def test_dense_small_all_three_edge_motifs(tm):
    g = ti.config_small_dense()
    say("dense_small_36")
    G = load(tm, g)
    mot = ti.three_edge_motifs()
    got = tm.count_exact_multi(G, mot, 3600)
    for M, c in zip(mot, got):
        want, _ = oracle.count(g.src, g.dst, g.t, M, 3600, hist=False)
        assert c == want, M


def test_edge_cases(tm):
    say("edge_cases")
    # empty graph
    e = ti.Graph(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), 3)
    G = load(tm, e, device=False)
    assert tm.count_exact(G, ti.TRIANGLE, 10) == 0
    assert tm.estimate(G, ti.TRIANGLE, 10, 2, 0.5, 0) == 0.0
    # single edge, all self-loops, all ties
    one = ti.Graph(np.array([0], np.int32), np.array([1], np.int32), np.array([5], np.int64), 2)
    G = load(tm, one, device=False)
    assert tm.count_exact(G, ((0, 1),), 0) == 1
    loops = ti.Graph(np.arange(5, dtype=np.int32), np.arange(5, dtype=np.int32), np.arange(5, dtype=np.int64), 5)
    G = load(tm, loops, device=False)
    assert tm.count_exact(G, ((0, 1),), 10) == 0
    ties = ti.Graph(np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32), np.array([7, 7, 7], np.int64), 3)
    G = load(tm, ties, device=False)
    assert tm.count_exact(G, ti.TRIANGLE, 10) == 0
    # negative and huge times, delta = infinity
    big = ti.Graph(np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32),
                   np.array([-(1 << 61), 0, (1 << 62)], np.int64), 3)
    G = load(tm, big, device=False)
    span = (1 << 62) + (1 << 61)
    assert tm.count_exact(G, ti.TRIANGLE, (1 << 63) - 1) == 1
    assert tm.count_exact(G, ti.TRIANGLE, span) == 1
    assert tm.count_exact(G, ti.TRIANGLE, span - 1) == 0


def test_errors(tm):
    say("errors")
    g = ti.random_small_graph(4, 50, 100, 1)
    G = load(tm, g, device=False)
    with pytest.raises(tm.TMError) as e:
        tm.count_exact(G, ((0, 1), (2, 3)), 5)
    assert e.value.status == 2  # not prefix-connected
    with pytest.raises(tm.TMError) as e:
        tm.count_exact(G, ((0, 2),), 5)
    assert e.value.status == 1  # not canonical
    with pytest.raises(tm.TMError) as e:
        tm.count_exact(G, ((0, 1), (1, 1)), 5)
    assert e.value.status == 1  # self-loop
    for (c, p) in ((1, 0.5), (2, 0.0), (2, 1.5), (2, float("nan"))):
        with pytest.raises(tm.TMError) as e:
            tm.estimate(G, ti.TRIANGLE, 5, c, p, 0)
        assert e.value.status == 1
    with pytest.raises(tm.TMError) as e:
        tm.load_graph(np.array([0, 7], np.int32), np.array([1, 1], np.int32), np.array([1, 2], np.int64), 4)
    assert e.value.status == 1


def test_per_anchor_counts(tm):
    g = ti.random_small_graph(6, 800, 2000, 77, allow_self_loops=True)
    say("per_anchor")
    G = load(tm, g)
    rng = np.random.default_rng(0)
    anchors = rng.choice(g.m, size=100, replace=False)
    win = rng.integers(0, 2500, size=100)
    for M in (ti.TRIANGLE, ti.STAR4, ti.BIFAN, ((0, 1), (1, 0), (0, 1)), ((0, 1),), ((0, 1), (1, 2))):
        got = tm.count_anchors(G, M, 50, anchors, win_end=win)
        want = oracle.count_anchors(g.src, g.dst, g.t - g.t.min(), M, 50, anchors, win_hi=win)
        assert (got == want).all()


THREE = ti.three_edge_motifs()


def test_sweep_estimates_all_three_edge_motifs(tm):
    """Estimates without diagnostics take the sweep counter (52-bit fixed-point
    weights, exact integer sums); they match the oracle's FP64 value."""
    g = ti.random_small_graph(6, 1200, 6000, 41, allow_self_loops=True)
    say("sweep_estimates")
    G = load(tm, g)
    for (delta, c, p, seed) in ((40, 2, 0.5, 3), (60, 3, 1.0, 4), (25, 10, 0.3, 5)):
        zs, kept = tm.estimate_multi(G, THREE, delta, c, p, seed)
        for M, z, k in zip(THREE, zs, kept):
            o = oracle.estimate(g.src, g.dst, g.t, M, delta, c, p, seed)
            assert close(z, o["Z"]), (M, z, o["Z"])
            assert k == int(o["win_counts"].sum()), M
        for M in THREE[::5]:
            assert close(tm.estimate(G, M, delta, c, p, seed), oracle.estimate(
                g.src, g.dst, g.t, M, delta, c, p, seed)["Z"])


def _one_triangle_graph(seed):
    """Nodes 0, 1, 2 only: many parallel edges of both directions on each of
    the three pairs, with tied times, so every role and direction of every
    triangle code occurs, plus a pendant pair without triangles."""
    rng = np.random.default_rng(seed)
    m = 900
    pairs = np.array([(0, 1), (1, 2), (0, 2), (2, 3)])
    k = rng.integers(0, 4, m)
    flip = rng.integers(0, 2, m).astype(bool)
    src = np.where(flip, pairs[k, 1], pairs[k, 0]).astype(np.int32)
    dst = np.where(flip, pairs[k, 0], pairs[k, 1]).astype(np.int32)
    t = (rng.integers(0, 300, m) * 3).astype(np.int64)  # ties
    return ti.Graph(src, dst, t, 4)


def test_static_triangles_equal_list_sweep(tm, monkeypatch):
    """The weighted triangle sums over the static triangles (the three pair
    timelines of each static triangle inside each kept window) and over the
    incidence lists are the same integers: every estimate and kept count of
    the 36 motifs is equal bit for bit, on bursty Zipf graphs with heavy
    pairs, a small multigraph, one-triangle graphs with tied times, a graph
    without any static triangle and a setting whose kept windows hold no
    triangle; the oracle checks the one-triangle cases."""
    cases = [
        (ti.config_zipf(200_000, 2_000, 1.8, 2_000_000, 7), 3600, 30, 0.1, 0),
        (ti.config_zipf(200_000, 2_000, 1.8, 2_000_000, 7), 3600, 10, 0.5, 3),
        (ti.config_zipf(100_000, 500, 1.5, 300_000, 8), 500, 3, 1.0, 1),
        (ti.random_small_graph(6, 1200, 6000, 41, allow_self_loops=True), 40, 2, 0.5, 3),
        (_one_triangle_graph(5), 40, 3, 0.7, 2),
        (_one_triangle_graph(6), 90, 2, 1.0, 4),
        # no static triangle at all (bipartite), and kept windows too few to hold one
        (ti.Graph(*(lambda r: (r.integers(0, 20, 3000).astype(np.int32), r.integers(20, 40, 3000).astype(np.int32),
                               r.integers(0, 50_000, 3000).astype(np.int64)))(np.random.default_rng(3)), 40),
         300, 3, 0.8, 5),
        (_one_triangle_graph(7), 40, 2, 1e-4, 6),
    ]
    for g, delta, c, p, seed in cases:
        say("static_triangles", g.m, g.n, delta, c, p, seed)
        G = load(tm, g)
        monkeypatch.setenv("TM_TRI_STATIC", "0")
        z0, k0 = tm.estimate_multi(G, THREE, delta, c, p, seed)
        monkeypatch.setenv("TM_TRI_STATIC", "1")  # also below the default size threshold
        z1, k1 = tm.estimate_multi(G, THREE, delta, c, p, seed)
        tm.profile_reset()
        tm.profile_enable(True)
        tm.estimate_multi(G, THREE, delta, c, p, seed)
        tm.profile_enable(False)
        if g.n != 40:  # the bipartite graph has no static triangle: nothing to launch
            assert tm.profile_read("tri_static_weight")[1] + tm.profile_read("tri_static_prep")[1] >= 1
        assert tm.profile_read("sweep3_tri_weight")[1] == 0
        monkeypatch.delenv("TM_TRI_STATIC")
        assert k1 == k0
        assert z1 == z0
        if g.n == 4 and p > 0.01:
            assert sum(k1[i] for i, M in enumerate(THREE) if len({x for e in M for x in e}) == 3) > 0
            for M, z, k in zip(THREE, z1, k1):
                o = oracle.estimate(g.src, g.dst, g.t, M, delta, c, p, seed)
                assert close(z, o["Z"]), (M, z, o["Z"])
                assert k == int(o["win_counts"].sum()), M


def test_static_triangles_huge_span(tm, monkeypatch):
    """Bursts of edges on four nodes at times up to 2^62: about 10^15 windows,
    far more than the per-call list of kept window ids holds, so each static
    triangle's walk draws every window its lightest pair touches.  Estimates
    and kept counts equal the incidence-list sweep's bit for bit."""
    rng = np.random.default_rng(9)
    pairs = np.array([(0, 1), (1, 2), (0, 2), (2, 3), (1, 3)])
    src, dst, t = [], [], []
    for base in (0, 1 << 40, 1 << 60, (1 << 62) - 5000):
        k = 300
        sel = rng.integers(0, len(pairs), k)
        flip = rng.integers(0, 2, k).astype(bool)
        src.append(np.where(flip, pairs[sel, 1], pairs[sel, 0]))
        dst.append(np.where(flip, pairs[sel, 0], pairs[sel, 1]))
        t.append(base + rng.integers(0, 4000, k))
    g = ti.Graph(np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32),
                 np.concatenate(t).astype(np.int64), 4)
    G = load(tm, g)
    tri_codes = [i for i, M in enumerate(THREE) if len({x for e in M for x in e}) == 3
                 and len({frozenset(e) for e in M}) == 3]
    kept_tri = 0
    for (delta, c, p, seed) in ((1000, 3, 0.6, 1), (500, 2, 1.0, 2), (2000, 5, 0.3, 3)):
        say("static_huge_span", delta, c, p, seed)
        monkeypatch.setenv("TM_TRI_STATIC", "0")
        z0, k0 = tm.estimate_multi(G, THREE, delta, c, p, seed)
        monkeypatch.setenv("TM_TRI_STATIC", "1")
        z1, k1 = tm.estimate_multi(G, THREE, delta, c, p, seed)
        monkeypatch.delenv("TM_TRI_STATIC")
        assert k1 == k0 and z1 == z0
        kept_tri += sum(k1[i] for i in tri_codes)
    assert kept_tri > 0


def test_static_triangles_per_window(tm, monkeypatch):
    """Edge-proportional estimates (b shifts, each kept window's weighted
    counts Y_{s,j} kept apart) with the triangle sums over the static
    triangles equal those over the incidence lists bit for bit: estimates,
    kept windows and every window's Y_{s,j}; the oracle checks the small
    case."""
    cases = [
        (ti.config_zipf(200_000, 2_000, 1.8, 2_000_000, 7), 3600, 10, 6.0, 3, 4),
        (_one_triangle_graph(8), 40, 2, 3.0, 2, 5),
    ]
    for g, delta, c, r, b, seed in cases:
        say("static_per_window", g.m, delta, c, r, b, seed)
        G = load(tm, g)
        monkeypatch.setenv("TM_TRI_STATIC", "0")
        e0, w0 = tm.estimate_q(G, THREE, delta, c, r, b, seed)
        monkeypatch.setenv("TM_TRI_STATIC", "1")
        e1, w1 = tm.estimate_q(G, THREE, delta, c, r, b, seed)
        monkeypatch.delenv("TM_TRI_STATIC")
        assert w0["n_kept"] == w1["n_kept"] > 0 and e0 == e1
        for key in ("k", "j", "q", "y"):
            assert np.array_equal(w0[key], w1[key]), key
        if g.n == 4:
            for i, M in enumerate(THREE):
                if len({x for e in M for x in e}) == 3 and len({frozenset(e) for e in M}) == 3:
                    o = oracle.estimate_q(g.src, g.dst, g.t, M, delta, c, r, b, seed)
                    assert close(e1[i], o["Z"]), (M, e1[i], o["Z"])


def test_static_triangles_not_kept_on_dense_graph(tm, monkeypatch):
    """A graph whose node pairs are nearly all joined has far more static
    triangles than edges: the index is not kept (the census reports the path
    as unsupported), and estimates, even with the static path forced, count
    triangles over the incidence lists, with the same results."""
    rng = np.random.default_rng(11)
    n, m = 300, 60_000
    src = rng.integers(0, n, m)
    dst = (src + rng.integers(1, n, m)) % n  # no self-loops
    g = ti.Graph(src.astype(np.int32), dst.astype(np.int32), np.sort(rng.integers(0, 2_000_000, m)).astype(np.int64),
                 n)
    say("static_not_kept", g.m, g.n)
    G = load(tm, g)
    with pytest.raises(tm.TMError) as e:
        tm.tri_static_census(G, 600, 3, 0.5, 1)
    assert e.value.status == 2
    monkeypatch.setenv("TM_TRI_STATIC", "0")
    z0, k0 = tm.estimate_multi(G, THREE, 600, 3, 0.5, 1)
    monkeypatch.setenv("TM_TRI_STATIC", "1")
    tm.profile_reset()
    tm.profile_enable(True)
    z1, k1 = tm.estimate_multi(G, THREE, 600, 3, 0.5, 1)
    tm.profile_enable(False)
    monkeypatch.delenv("TM_TRI_STATIC")
    assert z1 == z0 and k1 == k0
    assert tm.profile_read("sweep3_tri_weight")[1] == 1 and tm.profile_read("tri_static_weight")[1] == 0


def test_tri_static_census(tm):
    """The census of the static-triangle path counts, by brute force over the
    oracle's shift and kept windows: the (static triangle, kept window) units
    with edges on all three pairs in the window, and the (first, last) edge
    pairs on two pairs of a static triangle, in one kept window, within delta,
    with an edge of the third pair strictly between (the pairs the path
    visits); at least six tasks per unit (one per role)."""
    g = ti.random_small_graph(7, 400, 3000, 77)
    delta, c, p, seed = 60, 3, 0.6, 5
    say("tri_static_census", g.m, delta, c, p, seed)
    G = load(tm, g)
    o = oracle.estimate(g.src, g.dst, g.t, ti.TRIANGLE, delta, c, p, seed)
    s, L = int(o["s"]), c * delta
    kept = {int(j) for j in o["kept"]}
    t = (g.t - g.t.min()).astype(np.int64)
    win = (t - s) // L + 1
    pairs = {}
    for k, (u, v) in enumerate(zip(g.src.tolist(), g.dst.tolist())):
        if u != v:
            pairs.setdefault((min(u, v), max(u, v)), []).append(k)
    units = combos = 0
    for x in range(g.n):
        for y in range(x + 1, g.n):
            for z in range(y + 1, g.n):
                if (y, z) not in pairs or (x, z) not in pairs or (x, y) not in pairs:
                    continue
                P = [pairs[(y, z)], pairs[(x, z)], pairs[(x, y)]]
                common = set(win[P[0]]) & set(win[P[1]]) & set(win[P[2]]) & kept
                units += len(common)
                for r in range(3):
                    for i in range(3):
                        for j in range(3):
                            if len({i, j, r}) < 3:
                                continue
                            for a in P[i]:
                                if win[a] not in kept:
                                    continue
                                for e in P[j]:
                                    if win[e] != win[a] or not (t[a] < t[e] <= t[a] + delta):
                                        continue
                                    if any(t[a] < t[b] < t[e] for b in P[r]):
                                        combos += 1
    cen = tm.tri_static_census(G, delta, c, p, seed)
    assert units > 0 and combos > 0
    assert cen["units"] == units and cen["combos"] == combos, (cen, units, combos)
    assert cen["tasks"] >= 6 * units and cen["steps"] >= 1 and cen["triangles"] > 0


def test_estimate_q_matches_oracle(tm):
    """Algorithm 1 with b shifts and edge-proportional window probabilities
    (equation heuristic_q): the kept windows (shift, window, q_j) are the
    oracle's exactly; each window's weighted count Y_{s,j} and every motif's
    estimate agree within 1e-12."""
    cases = [
        (ti.random_small_graph(6, 1200, 6000, 51, allow_self_loops=True), 40, 3, 4.0, 3, 5, THREE),
        (ti.config_small_dense(2), 3600, 10, 8.0, 2, 9, THREE[::6]),
        (ti.random_small_graph(8, 3000, 20000, 52), 60, 2, 1e12, 1, 1, THREE[::5]),
    ]
    for g, delta, c, r, b, seed, motifs in cases:
        say("estimate_q", g.m, delta, c, r, b, seed)
        G = load(tm, g)
        est, win = tm.estimate_q(G, motifs, delta, c, r, b, seed)
        assert win["n_kept"] > 0
        for i, M in enumerate(motifs):
            o = oracle.estimate_q(g.src, g.dst, g.t, M, delta, c, r, b, seed)
            assert close(est[i], o["Z"]), (M, est[i], o["Z"])
            assert win["n_kept"] == o["n_kept"]
            assert np.array_equal(win["k"], o["k"]) and np.array_equal(win["j"], o["j"])
            assert np.array_equal(win["q"], o["q"])
            for y, yo in zip(win["y"][:, i], o["y"]):
                assert close(y, yo), (M, y, yo)
    # every non-empty window kept (r huge) with one shift: the p = 1 estimate
    g = ti.random_small_graph(7, 900, 4000, 53)
    G = load(tm, g)
    est, _ = tm.estimate_q(G, THREE, 30, 3, 1e12, 1, 4)
    est1, _ = tm.estimate_multi(G, THREE, 30, 3, 1.0, 4)
    for a, b_ in zip(est, est1):
        assert close(a, b_)


def test_estimate_q_four_edge_motifs(tm):
    """Edge-proportional estimates of four-edge motifs (generic counter per
    kept window, FP64 weighting of its duration histogram), alone and mixed
    with a three-edge motif: kept windows exactly the oracle's, Y_{s,j} and
    estimates within 1e-12."""
    cases = [
        (ti.zipf_graph(300, 4000, 1.5, 400_000, 61), 600, 4, 3.0, 3, 2, [ti.BIFAN, ti.CYCLE4, ti.STAR4]),
        (ti.random_small_graph(7, 1500, 5000, 62, allow_self_loops=True), 50, 3, 5.0, 2, 7,
         [ti.TRIANGLE, ti.CYCLE4]),
    ]
    for g, delta, c, r, b, seed, motifs in cases:
        say("estimate_q four-edge", g.m, delta, c, r, b, seed)
        G = load(tm, g)
        est, win = tm.estimate_q(G, motifs, delta, c, r, b, seed)
        assert win["n_kept"] > 0
        for i, M in enumerate(motifs):
            o = oracle.estimate_q(g.src, g.dst, g.t, M, delta, c, r, b, seed)
            assert close(est[i], o["Z"]), (M, est[i], o["Z"])
            assert win["n_kept"] == o["n_kept"]
            assert np.array_equal(win["k"], o["k"]) and np.array_equal(win["j"], o["j"])
            assert np.array_equal(win["q"], o["q"])
            for y, yo in zip(win["y"][:, i], o["y"]):
                assert close(y, yo), (M, y, yo)


def test_estimate_q_edge_cases(tm):
    g = ti.random_small_graph(5, 200, 1000, 54)
    G = load(tm, g)
    est, win = tm.estimate_q(G, THREE[:3], 20, 3, 2.0, 2, 0, cap=0)
    assert win["n_kept"] >= 0 and len(win["k"]) == 0
    est2, _ = tm.estimate_q(G, THREE[:3], 20, 3, 2.0, 2, 0)
    assert est == est2
    e = ti.Graph(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), 4)
    E = load(tm, e, device=False)
    z, w = tm.estimate_q(E, THREE[:2], 10, 2, 5.0, 3, 1)
    assert z == [0.0, 0.0] and w["n_kept"] == 0
    for bad in (dict(r=0.0), dict(r=-1.0), dict(r=float("inf")), dict(b=0), dict(c=1), dict(delta=0)):
        args = dict(delta=20, c=3, r=2.0, b=1)
        args.update(bad)
        with pytest.raises(tm.TMError):
            tm.estimate_q(G, THREE[:1], args["delta"], args["c"], args["r"], args["b"], 0)
    with pytest.raises(tm.TMError):  # the second edge touches no earlier node
        tm.estimate_q(G, [((0, 1), (2, 3), (0, 2), (1, 3))], 20, 3, 2.0, 1, 0)


def test_bifan_zipf(tm):
    """The bi-fan on a bursty Zipf graph (hubs, ties): exact counts with
    their duration histograms, and seed-matched estimates, against the
    oracle."""
    g = ti.zipf_graph(2000, 30000, 1.8, 200_000, 71)
    say("bifan_zipf", g.m)
    G = load(tm, g)
    for delta in (60, 600):
        got, hlo, hhi = tm.count_exact_multi(G, [ti.BIFAN], delta, hist=True)
        want, h = oracle.count(g.src, g.dst, g.t, ti.BIFAN, delta)
        assert got[0] == want, delta
        assert np.array_equal(hlo[0], h) and not hhi.any()
    for (c, p, seed) in ((10, 0.3, 1), (30, 1.0, 2)):
        z = tm.estimate(G, ti.BIFAN, 600, c, p, seed)
        o = oracle.estimate(g.src, g.dst, g.t, ti.BIFAN, 600, c, p, seed)
        assert close(z, o["Z"]), (c, p, seed, z, o["Z"])


STARS4 = [ti.STAR4, ((0, 1), (1, 0), (0, 2), (3, 0)), ((0, 1), (0, 1), (2, 1), (3, 1)), ((0, 1), (1, 0), (2, 1), (1, 3))]


def test_star4_counter(tm):
    """Four-edge stars whose first two edges share a leaf, through their own
    counter (running sums over the center's list, the heaviest 32 leaves of a
    node in LDS, the others from the pair timelines): exact counts,
    seed-matched estimates and their kept counts, and windowed counts against
    the oracle, on Zipf graphs whose hubs have hundreds of distinct leaves."""
    for g, delta, wins in ((ti.zipf_graph(300, 4000, 1.5, 400_000, 61), 600, ((50_000, 150_000),)),
                           (ti.zipf_graph(2000, 30000, 1.8, 200_000, 71), 300, ((20_000, 60_000),)),
                           (ti.random_small_graph(6, 900, 3000, 74, allow_self_loops=True), 80, ((500, 2000),))):
        say("star4", g.m, delta)
        G = load(tm, g)
        nl = g.src != g.dst
        nbrs = np.unique(np.concatenate([g.src[nl] * g.n + g.dst[nl], g.dst[nl] * g.n + g.src[nl]]))
        most = int(np.bincount(nbrs // g.n, minlength=g.n).max())  # distinct neighbours of the busiest node
        for M in STARS4:
            want, _ = oracle.count(g.src, g.dst, g.t, M, delta, hist=False)
            assert tm.count_exact(G, M, delta) == want, (M, delta)
            for (c, p, seed) in ((10, 0.5, 3), (3, 1.0, 1)):
                o = oracle.estimate(g.src, g.dst, g.t, M, delta, c, p, seed)
                z = tm.estimate(G, M, delta, c, p, seed)
                assert close(z, o["Z"]), (M, c, p, seed, z, o["Z"])
                zs, ks = tm.estimate_multi(G, [M, ti.TRIANGLE], delta, c, p, seed)
                assert zs[0] == z and ks[0] == int(o["win_counts"].sum())
            for (lo, hi) in wins:
                wc = tm.count_window(G, [M], delta, lo, hi)[0]
                assert wc == oracle.count(g.src, g.dst, g.t, M, delta, win=(lo, hi), hist=False)[0], (M, lo, hi)
        assert most > 32 or g.n <= 32  # the Zipf hubs take the light-leaf path


def test_estimate_stream_equals_in_memory(tm):
    """Streaming (kept windows in time order, one window's edges on the
    device at a time) gives the in-memory estimates and kept counts to the
    last bit, and the oracle's estimates within 1e-12, for three- and
    four-edge motifs; unsorted streams are refused."""
    cases = [
        (ti.random_small_graph(6, 1500, 8000, 81, allow_self_loops=True), 40, 3, 0.5, 2, True),
        (ti.config_small_dense(5), 3600, 10, 0.3, 1, True),
        (ti.zipf_graph(3000, 60000, 1.8, 2_000_000, 82), 3600, 5, 0.2, 3, False),
    ]
    for g, delta, c, p, seed, with_oracle in cases:
        say("estimate_stream", g.m, delta, c, p, seed)
        o = np.argsort(g.t, kind="stable")
        est, kc, info = tm.estimate_stream(g.src[o], g.dst[o], g.t[o], g.n, THREE, delta, c, p, seed)
        G = load(tm, g)
        e2, k2 = tm.estimate_multi(G, THREE, delta, c, p, seed)
        assert est == e2 and kc == k2
        assert info["n_kept"] > 0 and 0 < info["max_window_edges"] < g.m
        if with_oracle:
            for M, z in list(zip(THREE, est))[::9]:
                assert close(z, oracle.estimate(g.src, g.dst, g.t, M, delta, c, p, seed)["Z"]), M
        else:  # the Zipf graph: tier C, every motif at once
            o = oracle.estimate3_indexed(g.src, g.dst, g.t, THREE, delta, c, p, seed)
            assert o["n_kept"] == info["n_kept"] and o["s"] == info["shift"] and kc == o["kept_counts"]
            for M, z, zo in zip(THREE, est, o["Z"]):
                assert close(z, zo), (M, z, zo)
    g = ti.random_small_graph(5, 300, 1000, 83)
    assert not np.all(np.diff(g.t) >= 0)
    with pytest.raises(tm.TMError):
        tm.estimate_stream(g.src, g.dst, g.t, g.n, THREE[:1], 20, 3, 0.5, 0)
    z, k, info = tm.estimate_stream(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), 4,
                                    THREE[:2], 10, 2, 0.5, 0)
    assert z == [0.0, 0.0] and k == [0, 0] and info["n_kept"] == 0
    with pytest.raises(tm.TMError):  # the second edge touches no earlier node
        tm.estimate_stream(g.src[:1], g.dst[:1], g.t[:1], g.n, [((0, 1), (2, 3), (0, 2), (1, 3))], 20, 3, 0.5, 0)
    # four-edge motifs, alone and mixed with three-edge ones: tm_estimate's
    # value of each motif to the last bit, its kept count, and the oracle's
    for g, delta, c, p, seed, motifs in (
            (ti.zipf_graph(400, 6000, 1.5, 600_000, 85), 600, 4, 0.4, 3, [ti.BIFAN, ti.CYCLE4, ti.STAR4]),
            (ti.random_small_graph(7, 1500, 6000, 86, allow_self_loops=True), 50, 3, 0.5, 1,
             [ti.TRIANGLE, ti.CYCLE4, THREE[3]])):
        say("estimate_stream four-edge", g.m, delta, c, p, seed)
        o = np.argsort(g.t, kind="stable")
        est, kc, info = tm.estimate_stream(g.src[o], g.dst[o], g.t[o], g.n, motifs, delta, c, p, seed)
        assert info["n_kept"] > 0
        G = load(tm, g)
        _, k2 = tm.estimate_multi(G, motifs, delta, c, p, seed)
        assert kc == k2
        for M, z in zip(motifs, est):
            assert z == tm.estimate(G, M, delta, c, p, seed), M
            assert close(z, oracle.estimate(g.src, g.dst, g.t, M, delta, c, p, seed)["Z"]), M
    # device arrays are refused (the stream is read on the host)
    import ctypes
    s_dev, d_dev, t_dev = to_dev(ti.random_small_graph(5, 50, 1000, 84))
    m_ = int(t_dev.shape[0])
    arr = (tm.Motif * 1)(tm.motif(THREE[0]))
    est_ = (ctypes.c_double * 1)()
    rc = tm._lib.tm_estimate_stream(ctypes.c_void_p(s_dev.data_ptr()), ctypes.c_void_p(d_dev.data_ptr()),
                                    ctypes.c_void_p(t_dev.data_ptr()), m_, 5, 1, arr, 20, 3, 0.5, 0, est_, None,
                                    None, None)
    assert rc == 1  # TM_EINVAL


def test_two_node_pair_sweep(tm):
    """Weighted estimates of the four 2-node motifs alone take the sweep
    grouped by static edge; with a star motif added, the same motifs go
    through the per-node sweep.  Both sum exact fixed-point integers, so the
    estimates, kept counts and per-window Y_{s,j} agree to the last bit (one
    window per kept anchor, edge-proportional windows, streamed windows), and
    the oracle's estimates within 1e-12."""
    TWO = [M for M in THREE if len(set(sum(M, ()))) == 2]
    star = ((0, 1), (0, 1), (0, 2))
    cases = [
        (ti.random_small_graph(5, 1500, 6000, 91, allow_self_loops=True), 40, 3, 0.5, 2, True),
        (ti.zipf_graph(2000, 40000, 1.8, 2_000_000, 92), 86400, 3, 0.3, 1, False),
    ]
    for g, delta, c, p, seed, with_oracle in cases:
        say("two-node pair sweep", g.m, delta, c, p, seed)
        G = load(tm, g)
        e2, k2 = tm.estimate_multi(G, TWO, delta, c, p, seed)
        e3, k3 = tm.estimate_multi(G, TWO + [star], delta, c, p, seed)
        assert e2 == e3[:4] and k2 == k3[:4]
        assert any(k > 0 for k in k2)
        q2, w2 = tm.estimate_q(G, TWO, delta, c, 4.0, 2, seed)
        q3, w3 = tm.estimate_q(G, TWO + [star], delta, c, 4.0, 2, seed)
        assert q2 == q3[:4] and np.array_equal(w2["y"], w3["y"][:, :4])
        o = np.argsort(g.t, kind="stable")
        s2, ks2, _ = tm.estimate_stream(g.src[o], g.dst[o], g.t[o], g.n, TWO, delta, c, p, seed)
        assert s2 == e2 and ks2 == k2
        if with_oracle:
            for M, z in zip(TWO, e2):
                assert close(z, oracle.estimate(g.src, g.dst, g.t, M, delta, c, p, seed)["Z"]), M
        else:  # the Zipf graph at delta 86400: tier C
            o = oracle.estimate3_indexed(g.src, g.dst, g.t, TWO + [star], delta, c, p, seed)
            assert k3 == o["kept_counts"]
            for M, z, zo in zip(TWO + [star], e3, o["Z"]):
                assert close(z, zo), (M, z, zo)


def test_self_loop_only_graph(tm):
    """A graph whose edges are all self-loops holds no instance of any motif:
    every counter, estimator and the per-anchor counts give zero (the pair
    structures are empty)."""
    n, m = 6, 400
    rng = np.random.default_rng(95)
    u = rng.integers(0, n, m).astype(np.int32)
    g = ti.Graph(u, u.copy(), np.sort(rng.integers(0, 5000, m)).astype(np.int64), n)
    say("self-loop only", g.m)
    G = load(tm, g)
    assert G.n_pairs == 0
    ms = [ti.TRIANGLE, ((0, 1), (1, 0), (0, 1)), ti.BIFAN, ti.CYCLE4, ti.STAR4]
    got, hlo, hhi = tm.count_exact_multi(G, ms, 600, hist=True)
    assert all(c == 0 for c in got) and not hlo.any() and not hhi.any()
    est, kept = tm.estimate_multi(G, ms, 600, 3, 1.0, 0)
    assert est == [0.0] * len(ms) and kept == [0] * len(ms)
    q, w = tm.estimate_q(G, ms, 600, 3, 2.0, 2, 0)
    assert q == [0.0] * len(ms) and not np.any(w["y"])
    assert not np.any(tm.count_anchors(G, ti.CYCLE4, 600, np.arange(m)))


# kernels of an exact pass and of an estimate pass (its triangles over the
# static triangles: a set-up step, then the sums), and the incidence-list
# triangle kernel the estimate pass leaves out when the static path runs
SWEEP_NAMES = ("sweep3_fwd_count", "sweep3_tri_count", "sweep3_bwd_count",
               "sweep3_fwd_weight", "sweep3_bwd_weight", "tri_static_prep", "tri_static_weight")
UNUSED_NAMES = ("sweep3_tri_weight",)


def test_serial_timing_mode_same_results(tm, monkeypatch):
    """The serial timing mode (each pass's kernels one after another) changes
    how kernels run, never what they compute; in either mode every pass
    credits exactly one kernel as the one it waited for (the estimate pass
    with its triangles over the static triangles, forced on this small
    graph)."""
    monkeypatch.setenv("TM_TRI_STATIC", "1")
    g = ti.random_small_graph(6, 1200, 6000, 47, allow_self_loops=True)
    say("serial_timing")
    G = load(tm, g)
    runs = []
    try:
        for serial in (False, True):
            tm.profile_reset()
            tm.profile_enable(True, serial=serial)
            exact = tm.count_exact_multi(G, THREE, 40)
            est, kept = tm.estimate_multi(G, THREE, 40, 3, 0.5, 2)
            tm.profile_enable(False)
            crit = sum(tm.profile_read("crit:" + k)[1] for k in SWEEP_NAMES + UNUSED_NAMES)
            assert crit == 2, (serial, crit)  # one exact pass, one estimate pass
            assert all(tm.profile_read(k)[1] == 1 for k in SWEEP_NAMES), serial
            assert all(tm.profile_read(k)[1] == 0 for k in UNUSED_NAMES), serial
            runs.append((exact, est, kept))
    finally:
        tm.profile_enable(False)
    assert runs[0] == runs[1]
    for M, c in list(zip(THREE, runs[0][0]))[::7]:
        assert c == oracle.count(g.src, g.dst, g.t, M, 40, hist=False)[0], M


def test_count_window(tm):
    g = ti.random_small_graph(7, 1500, 8000, 43, allow_self_loops=True)
    say("count_window")
    G = load(tm, g)
    for (lo, hi) in ((1000, 2500), (0, 8000), (7990, 9000), (-50, 3)):
        for delta in (0, 30, 200):
            got = tm.count_window(G, THREE + [ti.CYCLE4, ti.STAR4], delta, lo, hi)
            for M, c in zip(THREE + [ti.CYCLE4, ti.STAR4], got):
                want, _ = oracle.count(g.src, g.dst, g.t, M, delta, win=(lo, hi), hist=False)
                assert c == want, (M, lo, hi, delta)


def test_exact_with_and_without_tables(tm):
    """Exact counts of all 36 three-edge motifs, whole-graph and windowed,
    from the exact-count tables (range sums) and from the window scans, each
    equal to the oracle's, on tie-heavy graphs with self-loops, repeated
    pairs and hubs."""
    cases = [(ti.random_small_graph(8, 1200, 2500, 71, allow_self_loops=True), (0, 9, 80)),
             (ti.random_small_graph(40, 3000, 40000, 72, allow_self_loops=False), (0, 500, 5000)),
             (ti.zipf_graph(300, 6000, 1.8, 50000, 73), (30, 3600))]
    for g, deltas in cases:
        say("tables", g.n, g.m)
        Gt = load(tm, g, exact_tables=True)
        Gs = load(tm, g, exact_tables=False)
        assert Gt.exact_table_bytes > 0 and Gs.exact_table_bytes == 0
        lo, hi = int(np.percentile(g.t, 30)), int(np.percentile(g.t, 70))
        for delta in deltas:
            a = tm.count_exact_multi(Gt, THREE, delta)
            b = tm.count_exact_multi(Gs, THREE, delta)
            wa = tm.count_window(Gt, THREE, delta, lo, hi)
            wb = tm.count_window(Gs, THREE, delta, lo, hi)
            for k, M in enumerate(THREE):
                want, _ = oracle.count(g.src, g.dst, g.t, M, delta, hist=False)
                assert a[k] == want and b[k] == want, (M, delta, a[k], b[k], want)
                want, _ = oracle.count(g.src, g.dst, g.t, M, delta, win=(lo, hi), hist=False)
                assert wa[k] == want and wb[k] == want, (M, delta, wa[k], wb[k], want)


def _wide_star_graph():
    """Node 0 (a hub) meets 1500 distinct leaves once each in [0, 1500); node
    1501 meets the hub every 50 s and 400 random leaves: its windows are long
    and the hub's window holds more distinct neighbours than the weighted
    triangle sweep's per-wave map takes."""
    rng = np.random.default_rng(81)
    src, dst, t = [], [], []
    for leaf in range(1, 1501):
        src.append(0), dst.append(leaf), t.append(leaf - 1)
    for k in range(30):
        src.append(1501), dst.append(0), t.append(50 * k + 7)
    for leaf in rng.integers(1, 1501, 400):
        if rng.random() < 0.5:
            src.append(1501), dst.append(int(leaf)), t.append(int(rng.integers(0, 1500)))
        else:
            src.append(int(leaf)), dst.append(1501), t.append(int(rng.integers(0, 1500)))
    perm = rng.permutation(len(src))
    return ti.Graph(np.array(src, np.int32)[perm], np.array(dst, np.int32)[perm], np.array(t, np.int64)[perm], 1502)


def test_weighted_triangles_long_windows(tm):
    """The weighted and histogram triangle sums of anchors with long windows
    (the wave-cooperative path, and its fallback when the window of the
    anchor's other endpoint has too many distinct neighbours) equal the
    oracle's, estimate by estimate and bin by bin."""
    tri = [M for M in THREE if len({x for e in M for x in e}) == 3 and
           not any(all(x in e for e in M) for x in range(3))]
    cases = [(ti.zipf_graph(1000, 20000, 1.6, 20000, 83), 600, (2, 1.0, 0), (5, 0.5, 3)),
             (_wide_star_graph(), 2000, (2, 1.0, 0), (3, 0.7, 5))]
    for g, delta, *settings in cases:
        say("long windows", g.n, g.m)
        G = load(tm, g)
        for c, p, seed in settings:
            got, _ = tm.estimate_multi(G, tri, delta, c, p, seed)
            for k, M in enumerate(tri):
                o = oracle.estimate(g.src, g.dst, g.t, M, delta, c, p, seed)
                assert close(got[k], o["Z"]), (M, c, p, seed, got[k], o["Z"])
        counts, hlo, hhi = tm.count_exact_multi(G, tri, delta, hist=True)
        for k, M in enumerate(tri):
            want, h = oracle.count(g.src, g.dst, g.t, M, delta, hist=True)
            assert counts[k] == want and (hhi[k] == 0).all() and (hlo[k] == h).all(), M


@pytest.mark.gpu
def test_generic_hist_both_bin_stores(tm):
    """Four-edge duration histograms on either side of the largest delta
    whose bins a block keeps in LDS (8192 bins): exact histograms and
    seed-matched estimates against the oracle."""
    g = ti.zipf_graph(500, 4000, 1.5, 2_000_000, 73)
    say("generic hist", g.m)
    G = load(tm, g)
    for delta in (8191, 8192, 20000):
        got, hlo, hhi = tm.count_exact_multi(G, [ti.BIFAN, ti.CYCLE4], delta, hist=True)
        for k, M in enumerate((ti.BIFAN, ti.CYCLE4)):
            want, h = oracle.count(g.src, g.dst, g.t, M, delta)
            assert got[k] == want and np.array_equal(hlo[k], h) and not hhi[k].any(), (M, delta)
        z = tm.estimate(G, ti.BIFAN, delta, 10, 0.5, 3)
        o = oracle.estimate(g.src, g.dst, g.t, ti.BIFAN, delta, 10, 0.5, 3)
        assert close(z, o["Z"]), (delta, z, o["Z"])
    # above the LDS bins an estimate without a histogram sums fixed-point
    # weights: the oracle's value, the histogram path's within 1e-12 and the
    # same kept count, and the streamed estimate to the last bit
    o_ = np.argsort(g.t, kind="stable")
    for delta in (8192, 20000):
        say("generic weighted sums", delta)
        est, kc, _ = tm.estimate_stream(g.src[o_], g.dst[o_], g.t[o_], g.n, [ti.CYCLE4, ti.BIFAN], delta, 10, 0.5, 3)
        for k, M in enumerate((ti.CYCLE4, ti.BIFAN)):
            z = tm.estimate(G, M, delta, 10, 0.5, 3)
            r = tm.estimate(G, M, delta, 10, 0.5, 3, info=True)
            o = oracle.estimate(g.src, g.dst, g.t, M, delta, 10, 0.5, 3)
            assert close(z, o["Z"]) and close(r["Z"], z), (M, delta, z, r["Z"], o["Z"])
            assert r["kept_count"] == int(o["win_counts"].sum()) == kc[k], (M, delta)
            assert est[k] == z, (M, delta, est[k], z)


@pytest.fixture(scope="module")
def zipf10m():
    return ti.config_zipf10m()


def test_zipf10m_heavy_windows(tm, zipf10m):
    """Full-size 10M-edge Zipf(1.8) graph: exact counts of the 36 three-edge
    motifs inside windows of two hours where the busiest node holds most
    edges (the per-window counting step), 2,000-3,000 edges and 20,000-40,000
    edges, against the oracle (tier C) on the same window sub-graphs."""
    g = zipf10m
    say("zipf10m windows: load")
    G = load(tm, g)
    delta = 3600
    tsort = np.sort(g.t)
    deg = np.bincount(g.src, minlength=g.n) + np.bincount(g.dst, minlength=g.n)
    hub = int(np.argmax(deg))
    on_hub = np.sort(g.t[(g.src == hub) | (g.dst == hub)])
    rng = np.random.default_rng(7)
    wins = {0: [], 1: []}
    for _ in range(20000):
        lo = int(rng.integers(0, 30_000_000 - 7200))
        hi = lo + 7199
        k = np.searchsorted(tsort, hi, side="right") - np.searchsorted(tsort, lo, side="left")
        kh = np.searchsorted(on_hub, hi, side="right") - np.searchsorted(on_hub, lo, side="left")
        if 2 * kh < k:
            continue
        if 2000 <= k <= 3000 and len(wins[0]) < 3:
            wins[0].append((lo, hi))
        if 20000 <= k <= 40000 and len(wins[1]) < 2:
            wins[1].append((lo, hi))
        if len(wins[0]) == 3 and len(wins[1]) == 2:
            break
    assert len(wins[0]) == 3 and len(wins[1]) == 2
    for (lo, hi) in wins[0] + wins[1]:
        sel = (g.t >= lo) & (g.t <= hi)
        say("zipf10m window", lo, hi, int(sel.sum()))
        got = tm.count_window(G, THREE, delta, lo, hi)
        want = oracle.count3_indexed(g.src[sel], g.dst[sel], g.t[sel], THREE, delta)
        assert got == want, (lo, hi)
        # the same window on its own: its exact counts, and the weighted sweep
        # with every edge in one kept window (p = 1), seed-matched
        sub = ti.Graph(g.src[sel], g.dst[sel], g.t[sel], g.n)
        Gw = load(tm, sub)
        assert tm.count_exact_multi(Gw, THREE, delta) == want
        c = 16  # the sub-graph spans at most 7,200 s: L = 57,600 holds it for most shifts
        seed = next(sd for sd in range(64) if oracle.draw(sd, 0, 0, 0) % (c * delta) <= c * delta - 7200)
        est, kept = tm.estimate_multi(Gw, THREE, delta, c, 1.0, seed)
        o = oracle.estimate3_indexed(sub.src, sub.dst, sub.t, THREE, delta, c, 1.0, seed)
        assert kept == o["kept_counts"] == want
        for M, z, zo in zip(THREE, est, o["Z"]):
            assert close(z, zo), (M, z, zo)
        Gw.free()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _check_golden(tm, G, ref):
    motifs = [tuple(tuple(e) for e in M) for M in ref["motifs"]]
    assert motifs == THREE
    delta = ref["delta"]
    got = tm.count_exact_multi(G, motifs, delta)
    assert got == [int(x) for x in ref["exact"]]
    for e in ref["estimates"]:
        say("golden estimate", e["c"], e["p"], e["seed"])
        est, kept = tm.estimate_multi(G, motifs, delta, e["c"], e["p"], e["seed"])
        assert kept == [int(x) for x in e["kept_counts"]], (e["c"], e["p"], e["seed"])
        for M, z, zo in zip(motifs, est, e["Z"]):
            assert close(z, zo), (M, e["c"], e["p"], e["seed"], z, zo)


def test_zipf_mid_config2_parameters(tm):
    """A 300k-edge graph drawn with the 10M-edge workload's recipe (Zipf 1.8,
    bursty, same edge density): exact counts of all 36 motifs and the
    estimates at c in {10, 30}, p in {0.01, 0.1}, seeds 0..7, against the
    oracle's stored values (tests/golden/make_zipf_mid_oracle.py)."""
    ref = _golden("zipf_mid_oracle.json")
    g = ti.zipf_graph(3000, 300_000, 1.8, 900_000, 12)
    say("zipf mid", g.m)
    G = load(tm, g)
    _check_golden(tm, G, ref)
    # kept windows and shift of one motif's diagnostics, seed by seed
    for e in ref["estimates"][::5]:
        r = tm.estimate(G, ti.TRIANGLE, ref["delta"], e["c"], e["p"], e["seed"], info=True)
        assert r["s"] == e["s"] and r["J"] == e["J"] and list(r["kept"]) == e["kept"]


def test_zipf10m_golden(tm, zipf10m):
    """Full size, the benchmark's workload and launch configuration: the 36
    exact whole-graph counts and the seed-0 estimates at the four benchmark
    settings (every kept window, hub windows of up to 1.6e5 edges) against
    the oracle's stored values (tests/golden/make_zipf10m_oracle.py)."""
    path = os.path.join(GOLDEN, "zipf10m_oracle.json")
    if not os.path.exists(path):
        pytest.skip("oracle values of the 10M-edge workload not generated")
    ref = _golden("zipf10m_oracle.json")
    say("zipf10m golden: load")
    G = load(tm, zipf10m)
    _check_golden(tm, G, ref)


def test_zipf10m_sampled_anchors(tm, zipf10m):
    """Full size: per-anchor counts (generic counter) for sampled anchors,
    hub anchors included, against the oracle's per-anchor brute force."""
    g = zipf10m
    G = load(tm, g)
    rng = np.random.default_rng(11)
    deg = np.bincount(g.src, minlength=g.n) + np.bincount(g.dst, minlength=g.n)
    hub = int(np.argmax(deg))
    # anchors whose delta-window holds at most 4000 edges keep the brute force short
    tsort = np.sort(g.t)
    w = np.searchsorted(tsort, g.t + 3600, side="right") - np.searchsorted(tsort, g.t, side="left")
    ok = np.nonzero(w <= 4000)[0]
    hub_ok = ok[(g.src[ok] == hub) | (g.dst[ok] == hub)]
    anchors = np.concatenate([rng.choice(ok, 6, replace=False), rng.choice(hub_ok, 2, replace=False)])
    tn = g.t - g.t.min()
    for M in (ti.TRIANGLE, ti.TWO_NODE_ALT, ((0, 1), (0, 2), (0, 2))):
        say("zipf10m anchors", M)
        got = tm.count_anchors(G, M, 3600, anchors)
        want = oracle.count_anchors(g.src, g.dst, tn, M, 3600, anchors)
        assert (got == want).all(), (M, got, want)


def test_batched_estimates_match_per_seed(tm):
    """tm_estimate_batch (persistent work-stealing launch, hipGraph replay)
    gives every seed's estimate and kept count exactly as the oracle does;
    replays with new seeds and eager work in between stay correct."""
    import torch
    g = ti.random_small_graph(7, 1500, 9000, 61, allow_self_loops=True)
    say("batch")
    G = load(tm, g)
    delta, c, p = 40, 3, 0.3
    # 10 seeds x p >= 1: stored anchor values plus boundary sweeps;
    # 3 seeds x p < 1: every kept anchor swept
    # triangle, star C (swept backwards), 2-node, star B, star A
    for M in (ti.TRIANGLE, ((0, 1), (0, 2), (0, 2)), ti.TWO_NODE_ALT, ((0, 1), (0, 2), (0, 1)), ((0, 1), (0, 1), (0, 2))):
        for n_seeds, plan in ((10, "count_batch_stored"), (3, "count_batch")):
            for tile in (64, 0):
                for rep in range(3):
                    seeds = np.arange(n_seeds, dtype=np.uint64) + 100 * rep + 7
                    tm.profile_reset()
                    tm.profile_enable(True)
                    est, kept = tm.estimate_batch(G, M, delta, c, p, seeds, tile=tile)
                    tm.profile_enable(False)
                    assert tm.profile_read(plan)[1] == 1, (M, n_seeds, plan)
                    for k, sd in enumerate(seeds):
                        o = oracle.estimate(g.src, g.dst, g.t, M, delta, c, p, int(sd))
                        assert close(est[k], o["Z"]), (M, n_seeds, tile, rep, k, est[k], o["Z"])
                        assert kept[k] == int(o["win_counts"].sum())
                    # eager work between replays
                    torch.zeros(1 << 20, device="cuda").sum().item()
                    assert close(tm.estimate(G, M, delta, c, p, int(seeds[0])), est[0])
    t, b = tm.batch_config(G, ti.TRIANGLE, delta, c, p)
    assert t in (64, 256, 1024) and b in (8, 16)
    # released plans and stored values are rebuilt with the same results
    seeds = np.arange(10, dtype=np.uint64) + 7
    before, _ = tm.estimate_batch(G, ti.TRIANGLE, delta, c, p, seeds)
    tm.batch_release(G)
    tm.profile_reset()
    tm.profile_enable(True)
    after, _ = tm.estimate_batch(G, ti.TRIANGLE, delta, c, p, seeds)
    tm.profile_enable(False)
    assert tm.profile_read("batch_anchor_values")[1] == 1
    assert list(before) == list(after)
    # a four-edge motif takes the seed-by-seed path
    est, kept = tm.estimate_batch(G, ti.CYCLE4, delta, c, p, [1, 2])
    for k, sd in enumerate((1, 2)):
        assert close(est[k], oracle.estimate(g.src, g.dst, g.t, ti.CYCLE4, delta, c, p, sd)["Z"])


def test_mixed_queries_share_one_launch(tm):
    """Queries with different motifs, deltas, c, p and seeds on one graph:
    the three-edge ones run as estimators of one captured persistent launch,
    the four-edge ones through the generic counter; every estimate and kept
    count equals that query's single-call result to the last bit, and the
    oracle's within 1e-12."""
    rng = np.random.default_rng(17)
    for g, deltas in ((ti.random_small_graph(7, 2500, 9000, 65, allow_self_loops=True), (20, 40, 90)),
                      (ti.zipf_graph(1500, 30000, 1.8, 600_000, 66), (600, 3600))):
        say("mixed", g.m)
        G = load(tm, g)
        qs = []
        for _ in range(48):
            M = THREE[int(rng.integers(0, len(THREE)))] if rng.random() < 0.9 else ti.CYCLE4
            qs.append((M, int(rng.choice(deltas)), int(rng.choice([2, 3, 10, 30])), float(rng.choice([0.2, 0.5, 1.0])),
                       int(rng.integers(0, 1 << 40))))
        tm.profile_reset()
        tm.profile_enable(True)
        est, kept = tm.estimate_mixed(G, qs)
        tm.profile_enable(False)
        assert tm.profile_read("count_batch_mixed")[1] == 1
        for (M, d, c, p, sd), z, k in zip(qs, est, kept):
            if len(M) == 3:
                z1, k1 = tm.estimate_multi(G, [M], d, c, p, sd)
                assert z == z1[0] and k == k1[0], (M, d, c, p, sd)
            else:
                r = tm.estimate(G, M, d, c, p, sd, info=True)
                assert z == r["Z"] and k == r["kept_count"]
        for (M, d, c, p, sd), z in list(zip(qs, est))[:6]:
            o = oracle.estimate(g.src, g.dst, g.t, M, d, c, p, sd)
            assert close(z, o["Z"]), (M, d, c, p, sd, z, o["Z"])


def test_batched_estimates_concurrent_same_plan(tm):
    """Two host threads run tm_estimate_batch with the same key (graph,
    motif, delta, c, p, seeds count, tile) on streams of their own, and a
    third releases the cached plans meanwhile: every call returns its own
    seeds' estimates, equal to the single-call ones."""
    import threading
    import torch
    g = ti.random_small_graph(7, 3000, 20000, 64, allow_self_loops=True)
    say("batch concurrent")
    G = load(tm, g)
    delta, c, p, M = 40, 3, 0.4, ti.TRIANGLE
    sets = [np.arange(16, dtype=np.uint64) + 1000 * (k + 1) for k in range(6)]
    want = [[tm.estimate(G, M, delta, c, p, int(sd)) for sd in S] for S in sets]
    out = [None] * len(sets)
    err = []

    def run(k, st):
        try:
            with torch.cuda.stream(st):
                for _ in range(3):
                    e, _ = tm.estimate_batch(G, M, delta, c, p, sets[k], tile=64, stream=st)
                    out[k] = list(e)
        except Exception as x:  # reported below
            err.append(x)

    def release():
        try:
            for _ in range(5):
                tm.batch_release(G)
        except Exception as x:
            err.append(x)

    streams = [torch.cuda.Stream() for _ in sets]
    th = [threading.Thread(target=run, args=(k, streams[k])) for k in range(len(sets))]
    th.append(threading.Thread(target=release))
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not err, err
    for k in range(len(sets)):
        assert out[k] == want[k], k


def _lists(g):
    """Per-node combined lists in the device's order: time, then input
    position, then the source's entry first (self-loops left out)."""
    keep = g.src != g.dst
    x = np.concatenate([g.src[keep], g.dst[keep]]).astype(np.int64)
    y = np.concatenate([g.dst[keep], g.src[keep]]).astype(np.int64)
    t = np.concatenate([g.t[keep], g.t[keep]]).astype(np.int64) - int(g.t.min())
    idx = np.concatenate([np.nonzero(keep)[0], np.nonzero(keep)[0]])
    side = np.concatenate([np.zeros(int(keep.sum()), np.int64), np.ones(int(keep.sum()), np.int64)])
    order = np.lexsort((side, idx, t, x))
    return x[order], y[order], t[order]


def _pair_sizes(g):
    """Edges per unordered node pair (self-loops left out)."""
    keep = g.src != g.dst
    a = np.minimum(g.src[keep], g.dst[keep]).astype(np.int64)
    b = np.maximum(g.src[keep], g.dst[keep]).astype(np.int64)
    k, c = np.unique(a * (1 << 32) + b, return_counts=True)
    return dict(zip(k.tolist(), c.tolist()))


def _probes(n):
    """Probes of one binary search over n sorted entries: ceil(log2(n + 1))."""
    return int(n).bit_length()


def _scan_counts(tv, yv, a, end, x, sizes, per_lookup, per_change):
    """Lookups, pair changes and probes of anchor a (at node x) over entries
    (a, end): entries tied with the anchor's time and entries leading to its
    own node are left out; a pair change is a lookup whose node differs from
    the previous one.  A lookup costs per_lookup searches of the pair {y1, yj}
    and a change one probe plus per_change searches."""
    ys = yv[a + 1:end][(tv[a + 1:end] != tv[a]) & (yv[a + 1:end] != yv[a])]
    if not ys.size:
        return 0, 0, 0
    y1 = int(yv[a])
    probes = 0
    prev = None
    for yj in ys.tolist():
        n = sizes.get(min(y1, yj) * (1 << 32) + max(y1, yj), 0)
        if yj != prev:
            probes += 1 + per_change * _probes(n)
        probes += per_lookup * _probes(n)
        prev = yj
    return int(ys.size), 1 + int((ys[1:] != ys[:-1]).sum()), probes


def _census_numpy(g, delta):
    """Entries each exact sweep scans, counted on the host from the
    definition: per node, the time-sorted incidence list of its
    non-self-loop edges; the forward (backward) entries of an anchor are the
    later (earlier) entries of its list within delta; the ranked sublist
    keeps the entries whose other endpoint has a longer list (ties: larger
    id); lookups and pair changes as in _scan_counts, over ranked entries."""
    x, y, t = _lists(g)
    sizes = _pair_sizes(g)
    deg = np.bincount(x, minlength=g.n)
    fwd = bwd = 0
    for v in np.unique(x):
        tv = t[x == v]
        fwd += int((np.searchsorted(tv, tv + delta, side="right") - np.arange(tv.size) - 1).sum())
        bwd += int((np.arange(tv.size) - np.searchsorted(tv, tv - delta, side="left")).sum())
    hi = (deg[y] > deg[x]) | ((deg[y] == deg[x]) & (y > x))
    rf = lk = pc = pr = 0
    for v in np.unique(x[hi]):
        sel = (x == v) & hi
        tv, yv = t[sel], y[sel]
        ends = np.searchsorted(tv, tv + delta, side="right")
        rf += int((ends - np.arange(tv.size) - 1).sum())
        for a in range(tv.size):
            l, c, q = _scan_counts(tv, yv, a, ends[a], v, sizes, 2, 2)
            lk += l
            pc += c
            pr += q
    return {"anchors": int(x.size), "fwd_entries": fwd, "bwd_entries": bwd, "tri_anchors": int(hi.sum()),
            "tri_entries": rf, "tri_lookups": lk, "tri_pairs": pc, "tri_probes": pr}


def _census_est_numpy(g, delta, c, p, seed):
    """The estimate's census: anchors in kept windows (shift and kept windows
    from the oracle), entries inside the anchor's window within delta."""
    o = oracle.estimate(g.src, g.dst, g.t, ti.TRIANGLE, delta, c, p, seed)
    s, L, kept = int(o["s"]), int(o["L"]), set(int(j) for j in o["kept"])
    x, y, t = _lists(g)
    sizes = _pair_sizes(g)
    an = fwd = bwd = lk = pc = pr = 0
    for v in np.unique(x):
        tv, yv = t[x == v], y[x == v]
        for a in range(tv.size):
            jw = (int(tv[a]) - s) // L + 1
            if jw not in kept:
                continue
            wlo, whi = s + (jw - 1) * L, s + jw * L - 1
            an += 1
            end = int(np.searchsorted(tv, min(int(tv[a]) + delta, whi), side="right"))
            beg = int(np.searchsorted(tv, max(int(tv[a]) - delta, wlo), side="left"))
            fwd += end - a - 1
            bwd += a - beg
            l, cc, q = _scan_counts(tv, yv, a, end, v, sizes, 1, 1)
            lk += l
            pc += cc
            pr += q
    return {"anchors": an, "fwd_entries": fwd, "bwd_entries": bwd, "tri_anchors": an, "tri_entries": fwd,
            "tri_lookups": lk, "tri_pairs": pc, "tri_probes": pr}


@pytest.mark.gpu
def test_sweep_census_matches_host_count(tm):
    """The work census behind the roofline figures counts exactly the list
    entries each sweep scans and the triangle sweeps' pair lookups, for the
    exact pass and for an estimate's kept windows."""
    for g, delta in ((ti.random_small_graph(30, 4000, 20000, 5, allow_self_loops=True), 300),
                     (ti.zipf_graph(2000, 30000, 1.8, 200000, 9), 3600)):
        G = load(tm, g)
        got = tm.sweep_census(G, delta)
        want = _census_numpy(g, delta)
        assert got == want, (got, want)
        for c, p, seed in ((3, 0.5, 7), (10, 0.6, 2)):
            got = tm.sweep_census_est(G, delta, c, p, seed)
            want = _census_est_numpy(g, delta, c, p, seed)
            assert got == want, (c, p, seed, got, want)
