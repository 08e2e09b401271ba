"""The allocation-free estimate entry point (tm_estimate_multi_noalloc),
called through the C ABI: its device outputs equal tm_estimate_multi's to
the last bit on two calls in a row, the second with a smaller input (fewer
edges, fewer motifs, a smaller delta), and its limits are enforced."""
import ctypes

import numpy as np
import pytest

import oracle
import tm_inputs as ti

pytestmark = pytest.mark.gpu

THREE = ti.three_edge_motifs()


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_1810_00980_amd as tm
    return tm


def _call(tm, G, motifs, delta, c, p, seed):
    """One call through the C ABI; returns (estimates, kept counts) read back
    after the stream is synchronized."""
    import torch
    k = len(motifs)
    est = torch.full((k,), float("nan"), dtype=torch.float64, device="cuda")
    kept = torch.full((2 * k,), 7, dtype=torch.int64, device="cuda")
    arr = (tm.Motif * k)(*[tm.motif(M) for M in motifs])
    st = torch.cuda.current_stream().cuda_stream
    rc = tm._lib.tm_estimate_multi_noalloc(G.handle, k, arr, int(delta), int(c), float(p), int(seed),
                                           ctypes.c_void_p(est.data_ptr()), ctypes.c_void_p(kept.data_ptr()),
                                           ctypes.c_void_p(st))
    assert rc == 0, rc
    torch.cuda.synchronize()
    kv = kept.cpu().numpy().view(np.uint64)
    return est.cpu().tolist(), [(int(kv[2 * i + 1]) << 64) | int(kv[2 * i]) for i in range(k)]


def _graph(tm, g):
    import torch
    s, d, t = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (g.src, g.dst, g.t))
    return tm.load_graph(s, d, t, g.n)


def test_noalloc_matches_estimate_multi_twice(tm):
    big = ti.random_small_graph(7, 2500, 9000, 301, allow_self_loops=True)
    small = ti.random_small_graph(5, 600, 3000, 302, allow_self_loops=True)
    print("[case] noalloc first call", big.m, flush=True)
    Gb = _graph(tm, big)
    e1, k1 = _call(tm, Gb, THREE, 60, 3, 0.5, 11)
    r1, rk1 = tm.estimate_multi(Gb, THREE, 60, 3, 0.5, 11)
    assert e1 == r1 and k1 == rk1
    assert any(k > 0 for k in k1)
    for M, z in list(zip(THREE, e1))[::7]:
        o = oracle.estimate(big.src, big.dst, big.t, M, 60, 3, 0.5, 11)
        assert abs(z - o["Z"]) <= 1e-12 * max(1.0, abs(o["Z"])), (M, z, o["Z"])
    print("[case] noalloc second call (smaller)", small.m, flush=True)
    Gs = _graph(tm, small)
    sub = THREE[5:14]
    e2, k2 = _call(tm, Gs, sub, 25, 4, 0.7, 3)
    r2, rk2 = tm.estimate_multi(Gs, sub, 25, 4, 0.7, 3)
    assert e2 == r2 and k2 == rk2
    for M, z in zip(sub, e2):
        o = oracle.estimate(small.src, small.dst, small.t, M, 25, 4, 0.7, 3)
        assert abs(z - o["Z"]) <= 1e-12 * max(1.0, abs(o["Z"])), (M, z, o["Z"])
    # the 2-node motifs alone take the pair-grouped kernel
    two = [M for M in THREE if len(set(sum(M, ()))) == 2]
    e3, k3 = _call(tm, Gb, two, 60, 3, 0.5, 11)
    r3, rk3 = tm.estimate_multi(Gb, two, 60, 3, 0.5, 11)
    assert e3 == r3 and k3 == rk3


def test_noalloc_limits(tm):
    g = ti.random_small_graph(5, 200, 1000, 303)
    print("[case] noalloc limits", flush=True)
    G = _graph(tm, g)
    import torch
    est = torch.zeros(2, dtype=torch.float64, device="cuda")
    one = (tm.Motif * 1)(tm.motif(ti.TRIANGLE))
    four = (tm.Motif * 1)(tm.motif(ti.CYCLE4))
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ep = ctypes.c_void_p(est.data_ptr())
    # delta above the scratch array's capacity, a four-edge motif: unsupported
    assert tm._lib.tm_estimate_multi_noalloc(G.handle, 1, one, tm.NOALLOC_MAX_DELTA + 1, 2, 0.5, 0, ep, None, st) == 2
    assert tm._lib.tm_estimate_multi_noalloc(G.handle, 1, four, 60, 2, 0.5, 0, ep, None, st) == 2
    # bad arguments
    assert tm._lib.tm_estimate_multi_noalloc(G.handle, 1, one, 60, 1, 0.5, 0, ep, None, st) == 1
    assert tm._lib.tm_estimate_multi_noalloc(G.handle, 0, one, 60, 2, 0.5, 0, ep, None, st) == 1
    assert tm._lib.tm_estimate_multi_noalloc(G.handle, 1, one, 60, 2, 0.5, 0, None, None, st) == 1
    # the largest delta is accepted
    e, k = _call(tm, G, [ti.TRIANGLE], tm.NOALLOC_MAX_DELTA, 2, 1.0, 0)
    r, rk = tm.estimate_multi(G, [ti.TRIANGLE], tm.NOALLOC_MAX_DELTA, 2, 1.0, 0)
    assert e == r and k == rk
