"""Pins for the CPU oracle: values, closed forms, identities and a second brute
force that the paper and the mathematics fix independently of the oracle's own
code.  No GPU needed."""
import itertools
import math
import os
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

import oracle
import tm_inputs as ti

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def arr(edges):
    s = np.array([e[0] for e in edges], dtype=np.int32)
    d = np.array([e[1] for e in edges], dtype=np.int32)
    t = np.array([e[2] for e in edges], dtype=np.int64)
    return s, d, t


def ocount(edges, motif, delta, win=None):
    s, d, t = arr(edges)
    return oracle.count(s, d, t, motif, delta, win=win)


def hist_of(counter, delta):
    h = np.zeros(delta + 1, dtype=np.uint64)
    for k, v in counter.items():
        h[k] = v
    return h


# ------------------------------------------------------------------ Philox

def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    assert len(rows) == 3
    for r in rows:
        assert oracle.philox4x32_10(r[0:4], r[4:6]) == r[6:10]


def test_draw_layout_and_uniformity():
    # draw = (word1 << 32) | word0 of counter (lo j, hi j, k, domain), key = seed
    seed, j = 0x0123456789ABCDEF, (5 << 32) | 7
    w = oracle.philox4x32_10([7, 5, 0, 1], [0x89ABCDEF, 0x01234567])
    assert oracle.draw(seed, j, 0, 1) == (w[1] << 32) | w[0]
    # chi-square of the top 4 bits over 8000 draws (15 dof, 0.1% critical ~37.7)
    cnt = Counter(oracle.draw(3, jj, 0, 1) >> 60 for jj in range(8000))
    chi = sum((cnt[b] - 500) ** 2 / 500 for b in range(16))
    assert chi < 37.7


# ------------------------------------------------------------ hand fixtures

TRI = ti.TRIANGLE


def test_h1_single_triangle():
    e = [(0, 1, 1), (1, 2, 2), (2, 0, 3)]
    for delta in (2, 3, 10):
        n, h = ocount(e, TRI, delta)
        assert n == 1 and h[2] == 1
    assert ocount(e, TRI, 1)[0] == 0
    # a rotation of the times is still a cyclic triangle ...
    assert ocount([(0, 1, 2), (1, 2, 3), (2, 0, 1)], TRI, 10)[0] == 1
    # ... but a reversal or a swap of the last two edges is not
    assert ocount([(0, 1, 3), (1, 2, 2), (2, 0, 1)], TRI, 10)[0] == 0
    assert ocount([(0, 1, 1), (1, 2, 3), (2, 0, 2)], TRI, 10)[0] == 0


def test_h2_tied_times_never_share_an_instance():
    assert ocount([(0, 1, 1), (1, 2, 1), (2, 0, 2)], TRI, 10)[0] == 0
    assert ocount([(0, 1, 1), (1, 2, 2), (2, 0, 2)], TRI, 10)[0] == 0
    assert ocount([(0, 1, 1), (1, 2, 2), (2, 0, 3)], TRI, 10)[0] == 1


@pytest.mark.parametrize("nab,nbc,nca", [(1, 1, 1), (3, 2, 4), (5, 1, 2)])
def test_h3_blocks_multiply(nab, nbc, nca):
    e, t = [], 0
    for (u, v, k) in ((0, 1, nab), (1, 2, nbc), (2, 0, nca)):
        for _ in range(k):
            t += 1
            e.append((u, v, t))
    assert ocount(e, TRI, t)[0] == nab * nbc * nca


def test_h4_single_pair_closed_form():
    Lc = 9
    e = [(0, 1, t) for t in range(1, Lc + 1)]
    m3 = ((0, 1), (0, 1), (0, 1))
    assert ocount(e, m3, Lc - 1)[0] == math.comb(Lc, 3)
    for delta in range(0, Lc + 1):
        expect = sum(math.comb(min(Lc - i, delta), 2) for i in range(1, Lc + 1))
        n, h = ocount(e, m3, delta)
        assert n == expect
        # durations: instance (i, j, k) has duration k - i; count per duration d
        # = (d - 1) middles times (Lc - d) anchors
        for d in range(delta + 1):
            assert int(h[d]) == (max(d - 1, 0) * (Lc - d) if d >= 2 else 0)


def test_h5_ex23_off_by_one_reading():
    e = [(0, 1, 1), (1, 0, 2), (0, 1, 3)]
    assert ocount(e, ti.TWO_NODE_ALT, 5)[0] == 1
    c = oracle.ex23(e, 5)
    assert sum(c.values()) == 1 and c[2] == 1


def test_h6_fig1_fragment():
    edges, motif, cases = [], None, []
    with open(os.path.join(GOLDEN, "fig1_fragment.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            p = line.split()
            if p[0] == "motif":
                v = [int(x) for x in p[1:]]
                motif = tuple(zip(v[0::2], v[1::2]))
            elif len(p) == 3 and p[2] != "-" and len(edges) < 4:
                edges.append(tuple(int(x) for x in p))
            else:
                cases.append((int(p[0]), int(p[1]), None if p[2] == "-" else int(p[2])))
    assert len(edges) == 4 and motif == ti.STAR4 and len(cases) == 4
    for delta, n_exp, dur in cases:
        n, h = ocount(edges, motif, delta)
        assert n == n_exp
        if dur is not None:
            assert h[dur] == 1


@pytest.mark.parametrize("d,k", [(5, 2), (6, 3), (7, 4), (4, 4)])
def test_h7_static_star_binomial(d, k):
    e = [(0, 1 + i, 1 + i) for i in range(d)]
    motif = tuple((0, 1 + j) for j in range(k))
    assert ocount(e, motif, d - 1)[0] == math.comb(d, k)
    assert ocount(e, motif, k - 2)[0] == 0


def test_h8_bijection_trap():
    e = [(0, 1, 1), (1, 0, 2), (0, 1, 3)]
    assert ocount(e, TRI, 10)[0] == 0
    # the same edges are one instance of the two-node motif
    assert ocount(e, ti.TWO_NODE_ALT, 10)[0] == 1


def test_h9_window_boundaries_every_shift():
    # delta = 5, c = 2 -> L = 10; the triangle spans times 8..12 (Delta = 4)
    e = [(0, 1, 0), (5, 6, 8), (6, 7, 10), (7, 5, 12), (3, 4, 25)]
    s, d, t = arr(e)
    delta, c = 5, 2
    L = c * delta
    for shift in range(-L + 1, 1):
        r = oracle.estimate(s, d, t, TRI, delta, c, 1.0, 0, force_shift=shift)
        # the instance is inside window j iff [8, 12] is inside [s+(j-1)L, s+jL-1]
        inside = any(shift + (j - 1) * L <= 8 and 12 <= shift + j * L - 1 for j in range(1, r["J"] + 1))
        assert int(r["win_counts"].sum()) == (1 if inside else 0)
        assert r["J"] == 1 + -(-25 // L)


# ------------------------------------------------- second brute force (tier B)

MOTIFS = ti.three_edge_motifs() + [ti.CYCLE4, ti.STAR4, ti.OUTSTAR5, ti.BIFAN, ((0, 1),), ((0, 1), (1, 0)),
                                    ((0, 1), (2, 0)), ((0, 1), (1, 2), (2, 3))]


@pytest.mark.parametrize("seed", range(6))
def test_tier_a_equals_tuple_brute_force(seed):
    g = ti.random_small_graph(4 + seed % 2, 13, 10, seed, allow_self_loops=(seed % 3 == 0))
    edges = list(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()))
    for M in MOTIFS:
        for delta in (0, 2, 6):
            b = oracle.brute(edges, M, delta)
            n, h = ocount(edges, M, delta)
            assert n == sum(b.values()), (M, delta)
            assert (h == hist_of(b, delta)).all(), (M, delta)
            win = (2, 7)
            bw = oracle.brute(edges, M, delta, win=win)
            nw, hw = ocount(edges, M, delta, win=win)
            assert nw == sum(bw.values()) and (hw == hist_of(bw, delta)).all()


def test_three_edge_motif_catalogue():
    mot = ti.three_edge_motifs()
    assert len(mot) == 36
    two = [m for m in mot if len({x for e in m for x in e}) == 2]
    assert len(two) == 4
    # 3-node motifs: stars have one node on all three edges, the rest are triangles
    three = [m for m in mot if m not in two]
    star = [m for m in three if any(all(x in e for e in m) for x in range(3))]
    assert len(star) == 24 and len(three) - len(star) == 8
    assert ti.TRIANGLE in mot and ti.TWO_NODE_ALT in mot


@pytest.mark.parametrize("seed", range(8))
def test_ex23_equals_oracle(seed):
    rng = np.random.default_rng(100 + seed)
    m = 40
    src = rng.integers(0, 4, m)
    dst = (src + rng.integers(1, 4, m)) % 4
    t = rng.permutation(300)[:m]
    edges = list(zip(src.tolist(), dst.tolist(), t.tolist()))
    for delta in (10, 60, 300):
        c = {d: n for d, n in oracle.ex23(edges, delta).items() if n}
        n, h = oracle.count(src, dst, t, ti.TWO_NODE_ALT, delta)
        assert c == {d: int(v) for d, v in enumerate(h) if v}


# ------------------------------------------------------------- hardness

def hardness_instance(n, gedges, k):
    """Temporal graph and star motif of the reduction from k-Clique (Sec. 3).
    Graph nodes 1..n, center 0.  Motif nodes: center 0, leaves 1..k."""
    T = []
    B = n + 2
    for (u, v) in gedges:
        T.append((0, u, (v - 1) * B + u + 1))
        T.append((0, v, (u - 1) * B + v + 1))
    for u in range(1, n + 1):
        T.append((u, 0, (u - 1) * B + 1))
        T.append((u, 0, u * B))
    S = []
    for leaf in range(1, k + 1):
        S.append((leaf, 0))
        S.extend((0, other) for other in range(1, k + 1) if other != leaf)
        S.append((leaf, 0))
    return T, tuple(S)


@pytest.mark.parametrize("seed", range(5))
def test_hardness_reduction_counts_cliques(seed):
    rng = np.random.default_rng(seed)
    n = 6
    gedges = [(u, v) for u in range(1, n + 1) for v in range(u + 1, n + 1) if rng.random() < 0.55]
    adj = set(gedges) | {(v, u) for u, v in gedges}
    for k in (2, 3):
        T, S = hardness_instance(n, gedges, k)
        s, d, t = arr(T)
        cnt, _ = oracle.count(s, d, t, S, oracle.INT64_MAX, hist=False)
        cliques = sum(1 for c in itertools.combinations(range(1, n + 1), k)
                      if all((a, b) in adj for a, b in itertools.combinations(c, 2)))
        assert cnt == cliques


# --------------------------------------------------- estimator identities

def small_cases():
    out = []
    for seed in range(4):
        g = ti.random_small_graph(4, 11, 14, 500 + seed)
        out.append(list(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist())))
    return out


@pytest.mark.parametrize("motif", [ti.TRIANGLE, ti.TWO_NODE_ALT, ((0, 1), (0, 2), (0, 1))])
@pytest.mark.parametrize("c", [2, 3])
def test_window_identities_every_shift(motif, c):
    """For every duration d: sum over all L shifts of the within-window
    histogram equals (L - d) * H(d)  (containment probability 1 - d/L), and
    the mean over shifts of ||Y_s||_1 equals C_M exactly (Lemma Ys_unbiased);
    the variance over shifts is at most C_M^2 / (c - 1) (Lemma var_Ys)."""
    delta = 3
    L = c * delta
    for edges in small_cases():
        H = oracle.brute(edges, motif, delta)
        CM = sum(H.values())
        per_s = oracle.windows_all_shifts(edges, motif, delta, c)
        assert len(per_s) == L
        tot = Counter()
        ys = []
        for s, wins in per_s.items():
            for w in wins:
                tot.update(w)
            ys.append(oracle.y_norm_exact(wins, L))
        for d in range(delta + 1):
            assert tot[d] == (L - d) * H[d]
        mean = sum(ys, Fraction(0)) / L
        assert mean == CM
        var = sum(((y - mean) ** 2 for y in ys), Fraction(0)) / L
        assert var <= Fraction(CM * CM, c - 1)
        # the C oracle's windowed counts agree with the tuple brute force
        s_, d_, t_ = arr(edges)
        for s in (-L + 1, -1, 0):
            r = oracle.estimate(s_, d_, t_, motif, delta, c, 1.0, 0, force_shift=s)
            assert r["n_kept"] == len(per_s[s])
            assert [int(x) for x in r["win_counts"]] == [sum(w.values()) for w in per_s[s]]
            # p = 1: Z equals ||Y_s||_1 for that shift
            y = oracle.y_norm_exact(per_s[s], L)
            assert abs(r["Z"] - float(y)) <= 1e-12 * max(1.0, float(y))


def test_p1_equals_norm_minus_straddlers():
    """At p = 1 the kept windows are all windows; their total equals C_M minus
    the instances that straddle a window boundary (exact integers)."""
    g = ti.random_small_graph(5, 60, 200, 77)
    edges = list(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()))
    s_, d_, t_ = arr(edges)
    delta, c = 20, 3
    L = c * delta
    tmin = int(t_.min())
    for seed in range(5):
        r = oracle.estimate(s_, d_, t_, ti.TRIANGLE, delta, c, 1.0, seed)
        sh = r["s"]
        win_of = lambda tt: (tt - tmin - sh) // L
        total, straddle = 0, 0
        for tup in itertools.permutations(range(len(edges)), 3):
            es = [edges[i] for i in tup]
            if not (es[0][2] < es[1][2] < es[2][2]) or es[2][2] - es[0][2] > delta:
                continue
            f = {}
            ok = True
            for (mu, mv), (gu, gv, _) in zip(ti.TRIANGLE, es):
                if f.setdefault(mu, gu) != gu or f.setdefault(mv, gv) != gv:
                    ok = False
            if not ok or len(set(f.values())) != 3:
                continue
            total += 1
            straddle += win_of(es[0][2]) != win_of(es[2][2])
        assert int(r["win_counts"].sum()) == total - straddle


def test_conditional_variance_lemma():
    """Lemma var_Zs: with the shift held fixed, Var[Z | s] = sum_j
    Y_{s,j}^2 (1/q_j - 1).  Closed form from exact per-window weights versus
    the empirical variance over 3000 seeds."""
    g = ti.random_small_graph(4, 70, 400, 9)
    edges = list(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()))
    s_, d_, t_ = arr(edges)
    delta, c, p = 15, 2, 0.3
    L = c * delta
    shift = -7
    tmin = int(t_.min())
    tn = t_ - tmin
    J = 1 + -(-int(tn.max()) // L)
    ys = []
    for j in range(1, J + 1):
        _, h = oracle.count(s_, d_, tn, ti.TWO_NODE_ALT, delta, win=(shift + (j - 1) * L, shift + j * L - 1))
        ys.append(sum(Fraction(int(n) * L, L - dd) for dd, n in enumerate(h) if n))
    ynorm = float(sum(ys))
    var_cf = float(sum(y * y for y in ys) * (1 / Fraction(p) - 1))
    assert var_cf > 0
    zs = np.array([oracle.estimate(s_, d_, t_, ti.TWO_NODE_ALT, delta, c, p, seed, force_shift=shift)["Z"]
                   for seed in range(3000)])
    assert abs(zs.mean() - ynorm) < 4 * math.sqrt(var_cf / len(zs))
    assert abs(zs.var() / var_cf - 1) < 0.12


def test_weight_matches_exact_rational():
    rng = np.random.default_rng(5)
    for delta, c, p in ((50, 2, 0.1), (3600, 30, 0.01), (7, 3, 1.0)):
        L = c * delta
        lo = rng.integers(0, 1 << 62, size=delta + 1, dtype=np.int64).astype(np.uint64)
        lo[rng.random(delta + 1) < 0.3] = 0
        hi = rng.integers(0, 4, size=delta + 1, dtype=np.int64).astype(np.uint64)
        z = oracle.weight(lo, delta, L, p, hist_hi=hi)
        exact = sum((Fraction((int(h) << 64) + int(l_) ) * Fraction(L, L - d) for d, (l_, h) in
                     enumerate(zip(lo, hi))), Fraction(0)) / Fraction(p)
        assert abs(Fraction(z) - exact) <= Fraction(1, 10 ** 12) * exact


@pytest.mark.slow
def test_estimator_unbiased_over_1000_seeds():
    """Mean of Z over seeds 0..999 lies within 3 standard errors of the exact
    count (the unbiasedness theorem of Sec. 4), on the 50-node version of the
    small uniform workload (triangle, delta 3600, c 30, p 0.1)."""
    g = ti.config_small_dense()
    delta, c, p = 3600, 30, 0.1
    CM, _ = oracle.count(g.src, g.dst, g.t, ti.TRIANGLE, delta, hist=False)
    assert CM > 100
    zs = np.array([oracle.estimate(g.src, g.dst, g.t, ti.TRIANGLE, delta, c, p, seed)["Z"]
                   for seed in range(1000)])
    se = zs.std(ddof=1) / math.sqrt(len(zs))
    assert abs(zs.mean() - CM) < 3 * se


# ------------------------------------------- edge-proportional q_j (Sec. 4)

def _window_edge_counts(t, shift, L):
    tn = np.asarray(t, dtype=np.int64) - int(np.min(t))
    J = 1 + -(-int(tn.max()) // L)
    return [int(((tn >= shift + (j - 1) * L) & (tn <= shift + j * L - 1)).sum()) for j in range(1, J + 1)]


def test_q_all_windows_kept_equals_p1():
    """With r so large that every non-empty window has q_j = 1, the
    edge-proportional estimate of one shift is ||Y_s||_1, the p = 1
    estimate of the same shift."""
    g = ti.config_small_dense(3)
    for seed in (0, 5):
        zq = oracle.estimate_q(g.src, g.dst, g.t, ti.TRIANGLE, 3600, 30, 1e12, 1, seed)
        zp = oracle.estimate(g.src, g.dst, g.t, ti.TRIANGLE, 3600, 30, 1.0, seed)
        assert np.all(zq["q"] == 1.0)
        assert abs(zq["Z"] - zp["Z"]) <= 1e-12 * zp["Z"]
        assert abs(zq["y"].sum() - zp["Z"]) <= 1e-12 * zp["Z"]


def test_q_window_weights_equal_tuple_brute_force():
    """Each kept window's Y_{s,j} equals the weighted count w(I_j) of Sec. 4
    computed exactly from the tier-B brute force restricted to the window."""
    g = ti.random_small_graph(5, 40, 300, 31)
    edges = list(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()))
    s_, d_, t_ = arr(edges)
    delta, c, shift = 20, 3, -17
    L = c * delta
    tmin = min(e[2] for e in edges)
    en = [(u, v, tt - tmin) for (u, v, tt) in edges]
    for motif in (ti.TRIANGLE, ti.TWO_NODE_ALT, ((0, 1), (0, 2), (0, 1))):
        r = oracle.estimate_q(s_, d_, t_, motif, delta, c, 1e12, 1, 0, force_shift=shift)
        assert r["n_kept"] > 0
        for j, y in zip(r["j"], r["y"]):
            h = oracle.brute(en, motif, delta, win=(shift + (j - 1) * L, shift + j * L - 1))
            exact = sum((Fraction(n * L, L - dd) for dd, n in h.items()), Fraction(0))
            assert abs(Fraction(y) - exact) <= Fraction(1, 10 ** 12) * max(exact, Fraction(1))


def test_q_probabilities_follow_window_edge_counts():
    """q_j = min(1, r |T_j| / |T|) with |T_j| counted from the times alone."""
    g = ti.config_small_dense(4)
    delta, c, r = 3600, 30, 1.5
    L = c * delta
    shift = -12345
    counts = _window_edge_counts(g.t, shift, L)
    res = oracle.estimate_q(g.src, g.dst, g.t, ti.TRIANGLE, delta, c, r, 1, 7, force_shift=shift)
    assert res["n_kept"] > 0
    for j, q in zip(res["j"], res["q"]):
        assert q == min(1.0, r * counts[j - 1] / g.m)


def test_q_conditional_mean_and_variance():
    """Lemma var_Zs with unequal q_j: with the shift fixed, E[Z | s] =
    ||Y_s||_1 and Var[Z | s] = sum_j Y_{s,j}^2 (1/q_j - 1); per-window
    weights from the counting oracle, q_j from the window edge counts,
    against 3000 seeds."""
    g = ti.random_small_graph(4, 70, 400, 9)
    s_, d_, t_ = g.src, g.dst, g.t
    delta, c, r, shift = 15, 2, 6.0, -7
    L = c * delta
    tn = t_ - int(t_.min())
    counts = _window_edge_counts(t_, shift, L)
    ys, qs = [], []
    for j in range(1, len(counts) + 1):
        _, h = oracle.count(s_, d_, tn, ti.TWO_NODE_ALT, delta, win=(shift + (j - 1) * L, shift + j * L - 1))
        ys.append(float(sum(Fraction(int(n) * L, L - dd) for dd, n in enumerate(h) if n)))
        qs.append(min(1.0, r * counts[j - 1] / g.m))
    ynorm = sum(ys)
    var_cf = sum(y * y * (1 / q - 1) for y, q in zip(ys, qs) if q > 0)
    assert var_cf > 0 and len(set(qs)) > 2
    zs = np.array([oracle.estimate_q(s_, d_, t_, ti.TWO_NODE_ALT, delta, c, r, 1, seed, force_shift=shift)["Z"]
                   for seed in range(3000)])
    assert abs(zs.mean() - ynorm) < 4 * math.sqrt(var_cf / len(zs))
    assert abs(zs.var() / var_cf - 1) < 0.12


def test_q_several_shifts_average():
    """Algorithm 1 returns the mean of the b per-shift sums; each shift k
    draws its own s and its own window uniforms."""
    g = ti.config_small_dense(1)
    res = oracle.estimate_q(g.src, g.dst, g.t, ti.TRIANGLE, 3600, 30, 2.0, 4, 11)
    per_k = [float(sum(y / q for k, y, q in zip(res["k"], res["y"], res["q"]) if k == kk)) for kk in range(4)]
    assert abs(res["Z"] - sum(per_k) / 4) <= 1e-12 * res["Z"]
    # the shifts differ: the kept window sets of the four shifts are not all equal
    sets = [tuple(res["j"][res["k"] == kk]) for kk in range(4)]
    assert len(set(sets)) > 1


@pytest.mark.slow
def test_q_estimator_unbiased_over_seeds():
    """Mean over 600 seeds of the b = 2, r = 2 estimate lies within 3
    standard errors of the exact count (unbiasedness of Sec. 4 with
    arbitrary q_j)."""
    g = ti.config_small_dense()
    delta, c = 3600, 30
    CM, _ = oracle.count(g.src, g.dst, g.t, ti.TRIANGLE, delta, hist=False)
    zs = np.array([oracle.estimate_q(g.src, g.dst, g.t, ti.TRIANGLE, delta, c, 2.0, 2, seed)["Z"]
                   for seed in range(600)])
    se = zs.std(ddof=1) / math.sqrt(len(zs))
    assert abs(zs.mean() - CM) < 3 * se


def test_bifan_is_canonical():
    assert ti.canonical(ti.BIFAN) == ti.BIFAN


def test_bifan_hand_example():
    """The bi-fan (0,1),(0,2),(3,1),(3,2): sources a, b and targets c, d
    with one edge per pair in motif order is one instance when its span fits
    delta; the same edges in another order, or a shared source, are none."""
    a, b, c, d = 0, 1, 2, 3
    one = [(a, c, 1), (a, d, 2), (b, c, 3), (b, d, 4)]
    assert ocount(one, ti.BIFAN, 3)[0] == 1
    assert ocount(one, ti.BIFAN, 2)[0] == 0
    swapped = [(a, c, 1), (b, c, 2), (a, d, 3), (b, d, 4)]
    assert ocount(swapped, ti.BIFAN, 10)[0] == 0
    same_source = [(a, c, 1), (a, d, 2), (a, c, 3), (a, d, 4)]
    assert ocount(same_source, ti.BIFAN, 10)[0] == 0
    # two parallel edges on every pair, all in motif order by blocks: 2^4 instances
    blocks = [(a, c, 1), (a, c, 2), (a, d, 3), (a, d, 4), (b, c, 5), (b, c, 6), (b, d, 7), (b, d, 8)]
    assert ocount(blocks, ti.BIFAN, 10)[0] == 16


# ------------------------------------------------------- per-anchor counts

@pytest.mark.parametrize("seed", range(4))
def test_per_anchor_counts_sum_to_total(seed):
    """orc_count_anchors over every edge adds up to orc_count's total and
    histogram (each instance has exactly one first edge)."""
    g = ti.random_small_graph(5 + seed, 160, 300, 40 + seed, allow_self_loops=True)
    allidx = np.arange(g.m)
    for M in (ti.TRIANGLE, ((0, 1), (0, 2), (0, 1)), ti.TWO_NODE_ALT, ti.CYCLE4, ti.STAR4, ((0, 1),),
              ((0, 1), (1, 0))):
        for delta in (0, 9, 60):
            per, h = oracle.count_anchors(g.src, g.dst, g.t, M, delta, allidx, hist=True)
            n, hw = oracle.count(g.src, g.dst, g.t, M, delta)
            assert int(per.sum(dtype=np.uint64)) == n, (M, delta)
            assert np.array_equal(h, hw), (M, delta)


@pytest.mark.parametrize("seed", range(4))
def test_per_anchor_counts_equal_tuple_brute_force(seed):
    """Per first edge, with and without a window end per anchor, against the
    tuple brute force filtered by first edge; the window bounds the first
    edge as well as the later ones."""
    g = ti.random_small_graph(4 + seed % 2, 12, 12, 300 + seed, allow_self_loops=(seed % 2 == 0))
    edges = list(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()))
    rng = np.random.default_rng(seed)
    win = rng.integers(-1, 14, g.m)
    allidx = np.arange(g.m)
    for M in (ti.TRIANGLE, ((0, 1), (0, 2), (0, 1)), ti.TWO_NODE_ALT, ti.CYCLE4, ((0, 1),), ((0, 1), (1, 2))):
        for delta in (0, 3, 8):
            b = oracle.brute_per_first(edges, M, delta)
            per = oracle.count_anchors(g.src, g.dst, g.t, M, delta, allidx)
            assert [int(x) for x in per] == [b[i] for i in range(g.m)], (M, delta)
            bw = oracle.brute_per_first(edges, M, delta, win_hi=win.tolist())
            perw = oracle.count_anchors(g.src, g.dst, g.t, M, delta, allidx, win_hi=win)
            assert [int(x) for x in perw] == [bw[i] for i in range(g.m)], (M, delta)


# ----------------------------------------------------------------- tier C

THREE = ti.three_edge_motifs()


@pytest.mark.parametrize("seed", range(10))
def test_tier_c_equals_tier_a(seed):
    """Tier C (every first/last pair sharing a node, middles by range counts)
    equals the brute force for all 36 motifs: counts and histograms, whole
    graph and windowed, on graphs with ties, repeated pairs and self-loops."""
    g = ti.random_small_graph(4 + seed % 5, 150 + 9 * seed, 400, 700 + seed, allow_self_loops=(seed % 2 == 0))
    for delta in (0, 5, 40, 1000):
        cnt, h = oracle.count3_indexed(g.src, g.dst, g.t, THREE, delta, hist=True, threads=2)
        for k, M in enumerate(THREE):
            want, hw = oracle.count(g.src, g.dst, g.t, M, delta)
            assert cnt[k] == want and np.array_equal(h[k], hw), (M, delta)
    for win in ((100, 250), (-5, 3), (390, 1000)):
        sub = THREE[3::4]
        cnt = oracle.count3_indexed(g.src, g.dst, g.t, sub, 40, win=win)
        for k, M in enumerate(sub):
            assert cnt[k] == oracle.count(g.src, g.dst, g.t, M, 40, win=win, hist=False)[0], (M, win)


@pytest.mark.parametrize("seed", range(4))
def test_tier_c_equals_tuple_brute_force(seed):
    g = ti.random_small_graph(4, 14, 9, 80 + seed, allow_self_loops=(seed % 2 == 1))
    edges = list(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()))
    for delta in (0, 2, 7):
        cnt, h = oracle.count3_indexed(g.src, g.dst, g.t, THREE, delta, hist=True)
        for k, M in enumerate(THREE):
            b = oracle.brute(edges, M, delta)
            assert cnt[k] == sum(b.values()) and np.array_equal(h[k], hist_of(b, delta)), (M, delta)


def test_tier_c_closed_forms():
    """Blocks n_ab n_bc n_ca of the cyclic triangle (H3) and C(L, 3) with the
    duration histogram (d - 1)(L - d) on one pair (H4), through tier C."""
    e, t = [], 0
    for (u, v, k) in ((0, 1, 7), (1, 2, 5), (2, 0, 9)):
        for _ in range(k):
            t += 1
            e.append((u, v, t))
    s, d, tt = arr(e)
    assert oracle.count3_indexed(s, d, tt, [TRI], t)[0] == 7 * 5 * 9
    Lc = 40
    s, d, tt = arr([(0, 1, x) for x in range(1, Lc + 1)])
    m3 = ((0, 1), (0, 1), (0, 1))
    cnt, h = oracle.count3_indexed(s, d, tt, [m3], Lc, hist=True)
    assert cnt[0] == math.comb(Lc, 3)
    assert [int(x) for x in h[0]] == [max(x - 1, 0) * (Lc - x) if x >= 2 else 0 for x in range(Lc + 1)]


def test_tier_c_thread_count_and_motif_order_do_not_matter():
    g = ti.zipf_graph(200, 5000, 1.5, 100_000, 5)
    a = oracle.count3_indexed(g.src, g.dst, g.t, THREE, 900, threads=1)
    b = oracle.count3_indexed(g.src, g.dst, g.t, THREE, 900, threads=5)
    c = oracle.count3_indexed(g.src, g.dst, g.t, THREE[::-1], 900, threads=3)
    assert a == b == c[::-1]
    with pytest.raises(oracle.OracleError):  # a repeated motif
        oracle.count3_indexed(g.src, g.dst, g.t, [TRI, TRI], 900)
    with pytest.raises(oracle.OracleError):  # not canonical
        oracle.count3_indexed(g.src, g.dst, g.t, [((1, 0), (0, 2), (2, 1))], 900)


def test_tier_c_estimate_equals_brute_force_estimate():
    """Algorithm 1 over tier C counts: the same shift, kept windows and, per
    motif, the same kept count and estimate (to the last bit: the same
    histogram weighted by the same routine) as the brute-force estimate."""
    g = ti.random_small_graph(6, 900, 5000, 31, allow_self_loops=True)
    for (delta, c, p, seed) in ((40, 2, 0.5, 1), (40, 3, 1.0, 2), (25, 10, 0.3, 3)):
        r = oracle.estimate3_indexed(g.src, g.dst, g.t, THREE, delta, c, p, seed, threads=2)
        for k, M in enumerate(THREE):
            o = oracle.estimate(g.src, g.dst, g.t, M, delta, c, p, seed)
            assert r["s"] == o["s"] and r["J"] == o["J"] and list(r["kept"]) == list(o["kept"])
            assert r["kept_counts"][k] == int(o["win_counts"].sum()), M
            assert r["Z"][k] == o["Z"], (M, r["Z"][k], o["Z"])


STARS4 = [ti.STAR4, ((0, 1), (1, 0), (0, 2), (3, 0)), ((0, 1), (0, 1), (2, 1), (3, 1)), ((0, 1), (1, 0), (2, 1), (1, 3))]


@pytest.mark.parametrize("seed", range(6))
def test_tier_c_stars_equal_tier_a(seed):
    """Tier C's four-edge stars (first three edges enumerated, the fourth by
    range counts) equal the brute force, whole graph and windowed, on graphs
    with ties, repeated pairs and self-loops."""
    g = ti.random_small_graph(5 + seed % 4, 160 + 10 * seed, 220, 900 + seed, allow_self_loops=(seed % 2 == 0))
    for M in STARS4:
        assert oracle.star4_directions(M) is not None
        for delta in (0, 12, 70, 1000):
            assert oracle.star4_indexed(g.src, g.dst, g.t, M, delta, threads=2) == \
                oracle.count(g.src, g.dst, g.t, M, delta, hist=False)[0], (M, delta)
        assert oracle.star4_indexed(g.src, g.dst, g.t, M, 40, win=(30, 160)) == \
            oracle.count(g.src, g.dst, g.t, M, 40, win=(30, 160), hist=False)[0], M


def test_tier_c_star_closed_form():
    """A center with n1 edges to leaf a at time 1, n2 more to a at time 2,
    n3 edges to each of k3 leaves at time 3 and n4 to each of k4 others at
    time 4: n1 n2 (n3 k3) (n4 k4) out-stars (0,1),(0,1),(0,2),(0,3)."""
    n1, n2, n3, k3, n4, k4 = 3, 4, 2, 3, 5, 2
    e = [(0, 1, 1)] * n1 + [(0, 1, 2)] * n2
    e += [(0, 2 + j, 3) for j in range(k3) for _ in range(n3)]
    e += [(0, 2 + k3 + j, 4) for j in range(k4) for _ in range(n4)]
    s, d, tt = arr(e)
    want = n1 * n2 * (n3 * k3) * (n4 * k4)
    assert oracle.star4_indexed(s, d, tt, ti.STAR4, 10) == want == oracle.count(s, d, tt, ti.STAR4, 10)[0]
