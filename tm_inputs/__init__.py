"""Seeded synthetic temporal graphs and motif query sets.

This module is the only code shared by the CPU oracle's tests and the HIP
path's tests and benchmarks.  It draws inputs; it holds none of the counting
or estimation arithmetic of the sampling framework.

A temporal graph is returned as three numpy arrays ``src`` (int32), ``dst``
(int32) and ``t`` (int64) of equal length ``m`` plus the node count ``n``.
Edges come out in generation order, which is NOT time order, so the device
sort is always exercised.

Generators (all seeded through numpy's PCG64):

* ``uniform_graph``: src uniform on {0..n-1}; dst uniform on the other n-1
  nodes (no self-loops); times uniform on {0..t_span-1}.
* ``zipf_graph``: src and dst drawn from Zipf(alpha) rank weights r^-alpha by
  inverse CDF, ranks mapped to ids through a seeded permutation (hubs carry no
  id locality), dst redrawn until it differs from src; times from
  ``bursty_times``.
* ``bursty_times``: an inhomogeneous Poisson process with a rate that is
  piecewise constant on one-hour bins, a daily sinusoid times a log-normal
  AR(1) burst factor; conditional on m the bin counts are multinomial and
  times are uniform inside a bin.

The temporal graphs stand in for the paper's ten public datasets (its
datasets table), which are not used here: only their shape (node count,
edge count, time span, one-second resolution, heavy-tailed degrees and
bursts) informs the recipes.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

HOUR = 3600


@dataclass(frozen=True)
class Graph:
    src: np.ndarray  # int32[m]
    dst: np.ndarray  # int32[m]
    t: np.ndarray    # int64[m]
    n: int

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_graph(n: int, m: int, t_span: int, seed: int) -> Graph:
    """Uniform endpoints without self-loops, uniform integer times in [0, t_span)."""
    if n < 2:
        raise ValueError("uniform_graph needs n >= 2")
    rng = _rng(seed)
    src = rng.integers(0, n, size=m, dtype=np.int64)
    dst = rng.integers(0, n - 1, size=m, dtype=np.int64)
    dst = dst + (dst >= src)
    t = rng.integers(0, t_span, size=m, dtype=np.int64)
    return Graph(src.astype(np.int32), dst.astype(np.int32), t, n)


def bursty_times(m: int, t_hi: int, rng: np.random.Generator, sigma: float = 1.5,
                 phi: float = 0.95, bin_s: int = HOUR,
                 gap_frac: float = 0.0) -> np.ndarray:
    """m integer times in [0, t_hi) from a bursty piecewise-constant-rate process.

    Rate of bin b: (1 + 0.5 sin(2 pi b / 24)) * exp(sigma G_b - sigma^2 / 2),
    G a stationary unit-variance AR(1) with coefficient phi.  With gap_frac > 0
    that fraction of bins (runs drawn from the same AR(1) field: the lowest
    values) gets rate zero, which creates empty stretches of time.
    """
    nb = (t_hi + bin_s - 1) // bin_s
    g = np.empty(nb)
    eps = rng.standard_normal(nb)
    g[0] = eps[0]
    c = np.sqrt(1.0 - phi * phi)
    for b in range(1, nb):
        g[b] = phi * g[b - 1] + c * eps[b]
    b_idx = np.arange(nb)
    lam = (1.0 + 0.5 * np.sin(2.0 * np.pi * b_idx / 24.0)) * np.exp(sigma * g - 0.5 * sigma * sigma)
    if gap_frac > 0.0:
        cut = np.quantile(g, gap_frac)
        lam[g <= cut] = 0.0
    # width of each bin (the last one may be partial)
    width = np.minimum(bin_s, t_hi - b_idx * bin_s)
    lam = lam * (width / bin_s)
    counts = rng.multinomial(m, lam / lam.sum())
    bins = np.repeat(b_idx, counts)
    off = (rng.random(m) * width[bins]).astype(np.int64)
    t = bins.astype(np.int64) * bin_s + off
    return t[rng.permutation(m)]


def _zipf_ids(n: int, alpha: float, size: int, rng: np.random.Generator,
              perm: np.ndarray, cdf: np.ndarray) -> np.ndarray:
    u = rng.random(size)
    r = np.searchsorted(cdf, u, side="right")
    r = np.minimum(r, n - 1)
    return perm[r]


def zipf_graph(n: int, m: int, alpha: float, t_hi: int, seed: int, sigma: float = 1.5,
               phi: float = 0.95, gap_frac: float = 0.0) -> Graph:
    """Zipf(alpha) endpoints (no self-loops), bursty times on [0, t_hi)."""
    if n < 2:
        raise ValueError("zipf_graph needs n >= 2")
    rng = _rng(seed)
    w = np.arange(1, n + 1, dtype=np.float64) ** (-alpha)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    perm = rng.permutation(n).astype(np.int64)
    src = _zipf_ids(n, alpha, m, rng, perm, cdf)
    dst = _zipf_ids(n, alpha, m, rng, perm, cdf)
    bad = np.nonzero(dst == src)[0]
    while bad.size:
        dst[bad] = _zipf_ids(n, alpha, bad.size, rng, perm, cdf)
        bad = bad[dst[bad] == src[bad]]
    t = bursty_times(m, t_hi, rng, sigma=sigma, phi=phi, gap_frac=gap_frac)
    return Graph(src.astype(np.int32), dst.astype(np.int32), t, n)


def zipf_graph_device(n: int, m: int, alpha: float, t_hi: int, seed: int, sigma: float = 1.5, phi: float = 0.95,
                      device: str = "cuda", chunk: int = 1 << 26):
    """The recipe of zipf_graph drawn on the GPU with torch's generator (for
    graphs of hundreds of millions of edges): returns device tensors src,
    dst (int32) and t (int64).  Endpoints: Zipf(alpha) ranks by inverse CDF
    through a seeded permutation of the ids, dst redrawn until it differs
    from src.  Times: the hourly rates of bursty_times (daily sinusoid times
    a log-normal AR(1) factor, drawn on the host from the same seed), each
    edge's hour drawn from them independently (the multinomial counts of
    bursty_times, without conditioning on m) and its offset uniform in the
    hour.  Edges come out in draw order, not time order."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    r = torch.arange(1, n + 1, dtype=torch.float64, device=device)
    cdf = torch.cumsum(r.pow(-alpha), 0)
    cdf /= cdf[-1].clone()
    del r
    perm = torch.randperm(n, generator=gen, device=device).to(torch.int32)

    def ids(size):
        out = torch.empty(size, dtype=torch.int32, device=device)
        for a in range(0, size, chunk):
            b = min(size, a + chunk)
            u = torch.rand(b - a, dtype=torch.float64, generator=gen, device=device)
            k = torch.searchsorted(cdf, u, right=True).clamp_(max=n - 1)
            out[a:b] = perm[k]
        return out

    src = ids(m)
    dst = ids(m)
    while True:
        bad = torch.nonzero(dst == src).flatten()
        if bad.numel() == 0:
            break
        dst[bad] = ids(bad.numel())
    # hourly rates from the host generator of the same seed
    rng = _rng(seed)
    nb = (t_hi + HOUR - 1) // HOUR
    g = np.empty(nb)
    eps = rng.standard_normal(nb)
    g[0] = eps[0]
    c = np.sqrt(1.0 - phi * phi)
    for b in range(1, nb):
        g[b] = phi * g[b - 1] + c * eps[b]
    b_idx = np.arange(nb)
    width = np.minimum(HOUR, t_hi - b_idx * HOUR)
    lam = (1.0 + 0.5 * np.sin(2.0 * np.pi * b_idx / 24.0)) * np.exp(sigma * g - 0.5 * sigma * sigma) * (width / HOUR)
    bcdf = torch.from_numpy(np.cumsum(lam) / lam.sum()).to(device)
    wid = torch.from_numpy(width).to(device)
    t = torch.empty(m, dtype=torch.int64, device=device)
    for a in range(0, m, chunk):
        b = min(m, a + chunk)
        u = torch.rand(b - a, dtype=torch.float64, generator=gen, device=device)
        k = torch.searchsorted(bcdf, u, right=True).clamp_(max=nb - 1)
        off = (torch.rand(b - a, dtype=torch.float64, generator=gen, device=device) * wid[k]).to(torch.int64)
        t[a:b] = k * HOUR + off
    return src, dst, t


def random_small_graph(n: int, m: int, t_span: int, seed: int, allow_self_loops: bool = False) -> Graph:
    """Tiny dense graphs with many repeated pairs and tied times (property tests)."""
    rng = _rng(seed)
    src = rng.integers(0, n, size=m, dtype=np.int64)
    if allow_self_loops:
        dst = rng.integers(0, n, size=m, dtype=np.int64)
    else:
        dst = rng.integers(0, n - 1, size=m, dtype=np.int64)
        dst = dst + (dst >= src)
    t = rng.integers(0, t_span, size=m, dtype=np.int64)
    return Graph(src.astype(np.int32), dst.astype(np.int32), t, n)


# ---------------------------------------------------------------- workloads

def config_small(seed: int = 0) -> Graph:
    """1,000 nodes, 20,000 uniform edges, times uniform on [0, 1e6)."""
    return uniform_graph(1000, 20000, 1_000_000, seed)


def config_small_dense(seed: int = 0) -> Graph:
    """The small workload with 50 nodes, so that triangle counts are non-zero."""
    return uniform_graph(50, 20000, 1_000_000, seed)


def config_zipf10m(seed: int = 2) -> Graph:
    """100k nodes, 10M edges, Zipf(1.8) endpoints, bursty times on [0, 3e7)."""
    return zipf_graph(100_000, 10_000_000, 1.8, 30_000_000, seed)


def config_batch50m(seed: int = 4) -> Graph:
    """500k nodes, 50M edges, Zipf(1.8), bursty times over [0, 3e8) with 30% of
    the hours silent: windows of 30 hours hold from tens to ~5e5 edges."""
    return zipf_graph(500_000, 50_000_000, 1.8, 300_000_000, seed, sigma=1.5, phi=0.95, gap_frac=0.3)


def config_zipf(m: int, n: int, alpha: float, t_hi: int, seed: int, **kw) -> Graph:
    return zipf_graph(n, m, alpha, t_hi, seed, **kw)


def config_star_cycle(device: str = "cuda"):
    """The four-edge workload: 20M nodes, 500M edges, Zipf(2.0) endpoints,
    bursty times over [0, 3e8) s (graph seed 3), drawn on the device."""
    return zipf_graph_device(20_000_000, 500_000_000, 2.0, 300_000_000, 3, device=device)


def serving_spec(i: int):
    """(n, m, t_hi, seed) of graph i (0..7) of the serving mix: 1e4 .. 1e8
    edges, log-spaced, 100 edges per node, Zipf(1.8) endpoints, bursty times
    over [0, max(1e6, 3m)) s."""
    m = int(round(10 ** (4 + 4 * i / 7)))
    return max(100, m // 100), m, max(1_000_000, 3 * m), 50 + i


def serving_graph(i: int) -> Graph:
    """Graph i (0..7) of the serving mix, drawn on the host."""
    n, m, t_hi, seed = serving_spec(i)
    return zipf_graph(n, m, 1.8, t_hi, seed)


def serving_graph_device(i: int, device: str = "cuda"):
    """Graph i of the serving mix drawn on the device (same recipe, torch's
    generator): src, dst, t tensors and n."""
    n, m, t_hi, seed = serving_spec(i)
    return (*zipf_graph_device(n, m, 1.8, t_hi, seed, device=device), n)


# ---------------------------------------------------------------- motifs

def canonical(edges):
    """Relabel motif nodes 0,1,2,... in order of first appearance."""
    lab = {}
    out = []
    for u, v in edges:
        for x in (u, v):
            if x not in lab:
                lab[x] = len(lab)
        out.append((lab[u], lab[v]))
    return tuple(out)


def three_edge_motifs():
    """All 36 connected 3-edge motifs on 2 or 3 nodes, canonical form, sorted.

    Enumerated from scratch: every sequence of three directed edges without
    self-loops over labels {0,1,2}, kept when it is connected and has at most
    3 nodes, deduplicated by first-appearance relabelling.  Returns 4 two-node
    and 32 three-node motifs.
    """
    pairs = [(u, v) for u in range(3) for v in range(3) if u != v]
    seen = set()
    for seq in itertools.product(pairs, repeat=3):
        c = canonical(seq)
        nodes = {x for e in c for x in e}
        # connected: every edge after the first touches an earlier node, or the
        # union graph is connected; with 3 edges on <= 3 nodes check union-find
        parent = {x: x for x in nodes}

        def find(x):
            while parent[x] != x:
                x = parent[x]
            return x
        for u, v in c:
            parent[find(u)] = find(v)
        if len({find(x) for x in nodes}) == 1:
            seen.add(c)
    return sorted(seen, key=lambda e: (len({x for p in e for x in p}), e))


TRIANGLE = ((0, 1), (1, 2), (2, 0))
TWO_NODE_ALT = ((0, 1), (1, 0), (0, 1))
CYCLE4 = ((0, 1), (1, 2), (2, 3), (3, 0))
STAR4 = ((0, 1), (0, 1), (0, 2), (0, 3))
OUTSTAR5 = ((0, 1), (0, 2), (0, 3), (0, 4))
# The bi-fan of the paper's second experiment (Sec. 5): two sources each
# linked to the same two targets.  The figure that fixed its edge order is
# lost, so this order (both edges of the first source, then both of the
# second, targets in the same order) is a reading; labels are canonical
# (numbered by first appearance): sources 0 and 3, targets 1 and 2.
BIFAN = ((0, 1), (0, 2), (3, 1), (3, 2))
