"""Python binding of libtm, the MI355X (gfx950) temporal-motif library.

Argument marshalling only: every step of counting and estimation runs in the
HIP kernels of ``libtm.so`` (built in-tree by ``build.py``).  The binding
raises ``ImportError`` when the library is missing, and ``TMError`` when a
call returns a status other than TM_OK; there is no CPU fallback.

Graph arrays can be numpy arrays (host) or torch tensors on the GPU (device);
torch is used only for device memory and the current stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libtm.so is not built ({LIB_PATH}); run paper_1810_00980_amd/build.py")

# A process holds one HIP runtime (torch's and the system's share the soname
# libamdhip64.so.7, and the first one loaded serves both).  Loading torch
# first makes it the one torch is built against, so that torch keeps its
# devices and the library shares its memory and streams.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIB_PATH)

STATUS = {0: "TM_OK", 1: "TM_EINVAL", 2: "TM_EUNSUPPORTED", 3: "TM_ENOMEM", 4: "TM_EBUDGET",
          5: "TM_EOVERFLOW", 6: "TM_EDEVICE"}


class TMError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({_lib.tm_strerror(status).decode()})")


class U128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]

    def value(self) -> int:
        return (int(self.hi) << 64) | int(self.lo)


class Motif(ctypes.Structure):
    _fields_ = [("l", ctypes.c_int32), ("src", ctypes.c_int32 * 4), ("dst", ctypes.c_int32 * 4)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("t_min", ctypes.c_int64),
                ("t_span", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("exact_table_bytes", ctypes.c_int64)]


class EstInfo(ctypes.Structure):
    _fields_ = [("shift", ctypes.c_int64), ("n_windows", ctypes.c_int64), ("n_kept", ctypes.c_int64),
                ("kept_count", U128), ("cap", ctypes.c_int64), ("kept_ids", ctypes.c_void_p),
                ("win_counts", ctypes.c_void_p), ("hist_lo", ctypes.c_void_p), ("hist_hi", ctypes.c_void_p)]


class QInfo(ctypes.Structure):
    _fields_ = [("n_kept", ctypes.c_int64), ("cap", ctypes.c_int64), ("win_k", ctypes.c_void_p),
                ("win_j", ctypes.c_void_p), ("win_q", ctypes.c_void_p), ("win_y", ctypes.c_void_p)]


class StreamInfo(ctypes.Structure):
    _fields_ = [("shift", ctypes.c_int64), ("n_windows", ctypes.c_int64), ("n_kept", ctypes.c_int64),
                ("max_window_edges", ctypes.c_int64), ("peak_graph_bytes", ctypes.c_int64)]


class Query(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("kind", ctypes.c_int32), ("motif", Motif), ("delta", ctypes.c_int64),
                ("c", ctypes.c_int64), ("p", ctypes.c_double), ("seed", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("count", U128), ("estimate", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double), ("batch_size", ctypes.c_int32),
                ("slot", ctypes.c_int32), ("ws_charged", ctypes.c_int64), ("ws_measured", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("wall_s", ctypes.c_double), ("edges_per_s", ctypes.c_double),
                ("budget_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("measured_max_bytes", ctypes.c_int64), ("over_charge", ctypes.c_int64),
                ("uncollected", ctypes.c_int64)]


P = ctypes.c_void_p
i64, i32, u64, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double

_SIGS = {
    "tm_load_graph": [P, P, P, i64, i32, i32, P, P],
    "tm_load_graph_ex": [P, P, P, i64, i32, ctypes.c_uint32, P, P],
    "tm_free_graph": [P],
    "tm_graph_info_get": [P, P],
    "tm_count_exact": [P, P, i64, P, P],
    "tm_count_exact_i64": [P, P, i64, P, P],
    "tm_count_exact_multi": [P, i32, P, i64, P, P, P, P],
    "tm_count_anchors": [P, P, i64, i64, P, P, P, P],
    "tm_count_window": [P, i32, P, i64, i64, i64, P, P],
    "tm_estimate": [P, P, i64, i64, f64, u64, P, P, P],
    "tm_estimate_multi": [P, i32, P, i64, i64, f64, u64, P, P, P],
    "tm_estimate_multi_noalloc": [P, i32, P, i64, i64, f64, u64, P, P, P],
    "tm_estimate_q": [P, i32, P, i64, i64, f64, i32, u64, P, P, P],
    "tm_estimate_stream": [P, P, P, i64, i32, i32, P, i64, i64, f64, u64, P, P, P, P],
    "tm_estimate_batch": [P, P, i64, i64, f64, i32, P, i32, P, P, P],
    "tm_batch_config": [P, P, i64, i64, f64, P, P, P],
    "tm_estimate_mixed": [P, i32, P, P, P, P],
    "tm_batch_release": [P, P],
    "tm_server_create": [i32, i64, P],
    "tm_server_add_graph": [P, P, P],
    "tm_server_submit": [P, P, P],
    "tm_server_wait": [P, i64, P],
    "tm_server_stats_get": [P, P],
    "tm_server_destroy": [P],
    "tm_profile_enable": [i32],
    "tm_profile_reset": [],
    "tm_profile_read": [ctypes.c_char_p, P, P],
    "tm_sweep_census": [P, i64, P, P],
    "tm_sweep_census_est": [P, i64, i64, f64, u64, P, P],
    "tm_tri_static_census": [P, i64, i64, f64, u64, P, P],
    "tm_strerror": [i32],
    "tm_version": [],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int32
_lib.tm_free_graph.restype = None
_lib.tm_server_destroy.restype = None
_lib.tm_strerror.restype = ctypes.c_char_p
_lib.tm_version.restype = ctypes.c_char_p

EXPORTED = tuple(_SIGS)


def _check(rc: int, what: str):
    if rc != 0:
        raise TMError(rc, what)


def _stream(stream=None):
    """A HIP stream handle: an integer handle, a torch stream, or (None) torch's
    current stream when torch has a GPU, else the null stream."""
    if stream is not None:
        if hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        return ctypes.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return ctypes.c_void_p(0)


def motif(edges) -> Motif:
    edges = tuple(tuple(e) for e in edges)
    if not 1 <= len(edges) <= 4:
        raise TMError(2, f"motif with {len(edges)} edges")
    m = Motif()
    m.l = len(edges)
    for i, (u, v) in enumerate(edges):
        m.src[i] = u
        m.dst[i] = v
    return m


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Graph:
    """A device-resident temporal graph (freed with the object)."""

    def __init__(self, src, dst, t, n_nodes: int, stream=None, exact_tables: bool = True):
        self._h = ctypes.c_void_p()
        self._keep = None
        on_device = 0
        if hasattr(src, "is_cuda") and src.is_cuda:
            import torch
            for a, dt in ((src, torch.int32), (dst, torch.int32), (t, torch.int64)):
                if a.dtype != dt or not a.is_contiguous():
                    raise TMError(1, "device arrays must be contiguous int32/int32/int64")
            ptrs = (src.data_ptr(), dst.data_ptr(), t.data_ptr())
            m = int(src.numel())
            on_device = 1
        else:
            s, d, tt = _np(src, np.int32), _np(dst, np.int32), _np(t, np.int64)
            if not (s.shape == d.shape == tt.shape):
                raise TMError(1, "src/dst/t lengths differ")
            self._keep = (s, d, tt)
            ptrs = (s.ctypes.data, d.ctypes.data, tt.ctypes.data)
            m = int(s.shape[0])
        flags = (1 if on_device else 0) | (0 if exact_tables else 2)
        _check(_lib.tm_load_graph_ex(P(ptrs[0]), P(ptrs[1]), P(ptrs[2]), m, int(n_nodes), flags,
                                     _stream(stream), ctypes.byref(self._h)), "tm_load_graph_ex")
        self._keep = None
        info = GraphInfo()
        _check(_lib.tm_graph_info_get(self._h, ctypes.byref(info)), "tm_graph_info_get")
        self.m, self.n, self.t_min, self.t_span = info.m, info.n, info.t_min, info.t_span
        self.n_pairs, self.device_bytes = info.n_pairs, info.device_bytes
        self.exact_table_bytes = info.exact_table_bytes

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h:
            _lib.tm_free_graph(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def load_graph(src, dst, t, n_nodes, stream=None, exact_tables: bool = True) -> Graph:
    return Graph(src, dst, t, n_nodes, stream, exact_tables)


def count_exact(g: Graph, edges, delta: int, stream=None) -> int:
    out = U128()
    _check(_lib.tm_count_exact(g.handle, ctypes.byref(motif(edges)), int(delta), ctypes.byref(out),
                               _stream(stream)), "tm_count_exact")
    return out.value()


def count_exact_i64(g: Graph, edges, delta: int, stream=None) -> int:
    out = ctypes.c_int64()
    _check(_lib.tm_count_exact_i64(g.handle, ctypes.byref(motif(edges)), int(delta), ctypes.byref(out),
                                   _stream(stream)), "tm_count_exact_i64")
    return int(out.value)


def count_exact_multi(g: Graph, motifs, delta: int, hist: bool = False, stream=None):
    k = len(motifs)
    arr = (Motif * max(k, 1))(*[motif(m) for m in motifs])
    cnt = (U128 * max(k, 1))()
    hlo = hhi = None
    if hist:
        hlo = np.zeros((k, delta + 1), dtype=np.uint64)
        hhi = np.zeros((k, delta + 1), dtype=np.uint64)
    _check(_lib.tm_count_exact_multi(g.handle, k, arr, int(delta), cnt,
                                     P(hlo.ctypes.data) if hist else None,
                                     P(hhi.ctypes.data) if hist else None, _stream(stream)),
           "tm_count_exact_multi")
    counts = [cnt[i].value() for i in range(k)]
    if hist:
        return counts, hlo, hhi
    return counts


def count_window(g: Graph, motifs, delta: int, t_lo: int, t_hi: int, stream=None):
    """Exact counts of each motif among edges with input time in [t_lo, t_hi]."""
    k = len(motifs)
    arr = (Motif * max(k, 1))(*[motif(m) for m in motifs])
    cnt = (U128 * max(k, 1))()
    _check(_lib.tm_count_window(g.handle, k, arr, int(delta), int(t_lo), int(t_hi), cnt, _stream(stream)),
           "tm_count_window")
    return [cnt[i].value() for i in range(k)]


def count_anchors(g: Graph, edges, delta: int, anchors, win_end=None, stream=None) -> np.ndarray:
    a = _np(anchors, np.int64)
    w = None if win_end is None else _np(win_end, np.int64)
    out = np.zeros(a.shape[0], dtype=np.uint64)
    _check(_lib.tm_count_anchors(g.handle, ctypes.byref(motif(edges)), int(delta), a.shape[0],
                                 P(a.ctypes.data), P(w.ctypes.data) if w is not None else None,
                                 P(out.ctypes.data), _stream(stream)), "tm_count_anchors")
    return out


def estimate(g: Graph, edges, delta: int, c: int, p: float, seed: int, info: bool = False,
             cap: int = 1 << 16, stream=None):
    z = ctypes.c_double()
    if not info:
        _check(_lib.tm_estimate(g.handle, ctypes.byref(motif(edges)), int(delta), int(c), float(p),
                                int(seed), ctypes.byref(z), None, _stream(stream)), "tm_estimate")
        return z.value
    kept = np.zeros(cap, dtype=np.int64)
    wc = np.zeros(cap, dtype=np.uint64)
    hlo = np.zeros(delta + 1, dtype=np.uint64)
    hhi = np.zeros(delta + 1, dtype=np.uint64)
    ei = EstInfo()
    ei.cap = cap
    ei.kept_ids, ei.win_counts = kept.ctypes.data, wc.ctypes.data
    ei.hist_lo, ei.hist_hi = hlo.ctypes.data, hhi.ctypes.data
    _check(_lib.tm_estimate(g.handle, ctypes.byref(motif(edges)), int(delta), int(c), float(p), int(seed),
                            ctypes.byref(z), ctypes.byref(ei), _stream(stream)), "tm_estimate")
    n = max(0, min(ei.n_kept, cap))
    return {"Z": z.value, "s": ei.shift, "J": ei.n_windows, "n_kept": ei.n_kept,
            "kept_count": ei.kept_count.value(), "kept": kept[:n].copy(), "win_counts": wc[:n].copy(),
            "hist_lo": hlo, "hist_hi": hhi}


def estimate_multi(g: Graph, motifs, delta: int, c: int, p: float, seed: int, stream=None):
    k = len(motifs)
    arr = (Motif * max(k, 1))(*[motif(m) for m in motifs])
    est = (ctypes.c_double * max(k, 1))()
    kc = (U128 * max(k, 1))()
    _check(_lib.tm_estimate_multi(g.handle, k, arr, int(delta), int(c), float(p), int(seed), est, kc,
                                  _stream(stream)), "tm_estimate_multi")
    return [est[i] for i in range(k)], [kc[i].value() for i in range(k)]


NOALLOC_MAX_DELTA = 1048575


def estimate_multi_noalloc(g: Graph, motifs, delta: int, c: int, p: float, seed: int, est_dev, kept_dev=None,
                           stream=None):
    """tm_estimate_multi_noalloc: the estimates of tm_estimate_multi written
    into caller-owned device buffers (est_dev: float64 tensor of len(motifs);
    kept_dev: nullable uint64 tensor of 2 len(motifs) words, lo/hi per motif)
    without any device allocation.  Returns once the work is enqueued on the
    stream; synchronize before reading the buffers."""
    k = len(motifs)
    arr = (Motif * max(k, 1))(*[motif(m) for m in motifs])
    _check(_lib.tm_estimate_multi_noalloc(g.handle, k, arr, int(delta), int(c), float(p), int(seed),
                                          P(est_dev.data_ptr()), P(kept_dev.data_ptr()) if kept_dev is not None
                                          else None, _stream(stream)), "tm_estimate_multi_noalloc")


def estimate_q(g: Graph, motifs, delta: int, c: int, r: float, b: int, seed: int, cap: int = 4096, stream=None):
    """Algorithm 1 with b shifts and window probabilities q_j = min(1, r |T_j| / |T|)
    (motifs of up to four edges).  Returns (estimates, windows): windows holds, for the
    first `cap` kept windows in order of (shift, window), arrays k, j, q and
    y (Y_{s,j} per motif, shape [windows, motifs]), and n_kept over all shifts."""
    k = len(motifs)
    arr = (Motif * max(k, 1))(*[motif(m) for m in motifs])
    est = (ctypes.c_double * max(k, 1))()
    wk = np.zeros(max(cap, 1), dtype=np.int64)
    wj = np.zeros(max(cap, 1), dtype=np.int64)
    wq = np.zeros(max(cap, 1), dtype=np.float64)
    wy = np.zeros((max(cap, 1), max(k, 1)), dtype=np.float64)
    info = QInfo(0, int(cap), wk.ctypes.data, wj.ctypes.data, wq.ctypes.data, wy.ctypes.data)
    _check(_lib.tm_estimate_q(g.handle, k, arr, int(delta), int(c), float(r), int(b), int(seed), est,
                              ctypes.byref(info), _stream(stream)), "tm_estimate_q")
    n = min(info.n_kept, cap)
    return [est[i] for i in range(k)], {"n_kept": info.n_kept, "k": wk[:n].copy(), "j": wj[:n].copy(),
                                        "q": wq[:n].copy(), "y": wy[:n, :k].copy()}


def estimate_stream(src, dst, t, n_nodes: int, motifs, delta: int, c: int, p: float, seed: int, stream=None):
    """Algorithm 1 over host arrays sorted by time, one kept window on the
    device at a time (motifs of up to four edges).  Returns (estimates, kept
    counts, info dict)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int64)
    m = int(t.shape[0])
    if src.shape[0] != m or dst.shape[0] != m:
        raise ValueError("src, dst and t differ in length")
    k = len(motifs)
    arr = (Motif * max(k, 1))(*[motif(x) for x in motifs])
    est = (ctypes.c_double * max(k, 1))()
    kc = (U128 * max(k, 1))()
    info = StreamInfo()
    _check(_lib.tm_estimate_stream(P(src.ctypes.data), P(dst.ctypes.data), P(t.ctypes.data), m, int(n_nodes), k,
                                   arr, int(delta), int(c), float(p), int(seed), est, kc, ctypes.byref(info),
                                   _stream(stream)), "tm_estimate_stream")
    return ([est[i] for i in range(k)], [kc[i].value() for i in range(k)],
            {"shift": info.shift, "n_windows": info.n_windows, "n_kept": info.n_kept,
             "max_window_edges": info.max_window_edges, "peak_graph_bytes": info.peak_graph_bytes})


def estimate_batch(g: Graph, edges, delta: int, c: int, p: float, seeds, tile: int = 0, stream=None):
    s = _np(seeds, np.uint64)
    k = s.shape[0]
    est = np.zeros(k, dtype=np.float64)
    kc = (U128 * max(k, 1))()
    _check(_lib.tm_estimate_batch(g.handle, ctypes.byref(motif(edges)), int(delta), int(c), float(p), k,
                                  P(s.ctypes.data), int(tile), P(est.ctypes.data), kc, _stream(stream)),
           "tm_estimate_batch")
    return est, [kc[i].value() for i in range(k)]


class EstQuery(ctypes.Structure):
    _fields_ = [("motif", Motif), ("delta", ctypes.c_int64), ("c", ctypes.c_int64), ("p", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


def estimate_mixed(g: Graph, queries, stream=None):
    """Estimates of queries [(motif edges, delta, c, p, seed)] on one graph,
    the three-edge ones in one launch.  Returns (estimates, kept counts)."""
    k = len(queries)
    arr = (EstQuery * max(k, 1))(*[EstQuery(motif(M), int(d), int(c), float(p), int(s))
                                   for (M, d, c, p, s) in queries])
    est = (ctypes.c_double * max(k, 1))()
    kc = (U128 * max(k, 1))()
    _check(_lib.tm_estimate_mixed(g.handle, k, arr, est, kc, _stream(stream)), "tm_estimate_mixed")
    return [est[i] for i in range(k)], [kc[i].value() for i in range(k)]


def profile_enable(on: bool = True, serial: bool = False):
    """Kernel timing on/off; serial=True also runs the kernels of each sweep
    pass one after another, so that each duration is the kernel's own."""
    _check(_lib.tm_profile_enable((2 if serial else 1) if on else 0), "tm_profile_enable")


def profile_reset():
    _check(_lib.tm_profile_reset(), "tm_profile_reset")


def profile_read(kernel: str):
    """(total milliseconds, launches) of a library kernel since the last reset."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(_lib.tm_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)), "tm_profile_read")
    return ms.value, n.value


class Census(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("anchors", "fwd_entries", "bwd_entries", "tri_anchors", "tri_entries", "tri_lookups", "tri_pairs",
                 "tri_probes")]


def sweep_census(g: Graph, delta: int, stream=None) -> dict:
    """Work census of the exact three-edge sweeps (tm_census fields)."""
    c = Census()
    _check(_lib.tm_sweep_census(g.handle, int(delta), ctypes.byref(c), _stream(stream)), "tm_sweep_census")
    return {name: getattr(c, name) for name, _ in Census._fields_}


def sweep_census_est(g: Graph, delta: int, c: int, p: float, seed: int, stream=None) -> dict:
    """Work census of an estimate's weighted sweeps (tm_census fields)."""
    r = Census()
    _check(_lib.tm_sweep_census_est(g.handle, int(delta), int(c), float(p), int(seed), ctypes.byref(r),
                                    _stream(stream)), "tm_sweep_census_est")
    return {name: getattr(r, name) for name, _ in Census._fields_}


class TriCensus(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in ("triangles", "units", "tasks", "drivers", "steps", "combos")]


def tri_static_census(g: Graph, delta: int, c: int, p: float, seed: int, stream=None) -> dict:
    """Work census of an estimate's weighted triangle sums over the static
    triangles (tm_tri_census fields)."""
    r = TriCensus()
    _check(_lib.tm_tri_static_census(g.handle, int(delta), int(c), float(p), int(seed), ctypes.byref(r),
                                     _stream(stream)), "tm_tri_static_census")
    return {name: getattr(r, name) for name, _ in TriCensus._fields_}


def batch_config(g: Graph, edges, delta: int, c: int, p: float, stream=None):
    """Autotuned (tile, work-groups per CU) of the batched estimator."""
    t, b = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.tm_batch_config(g.handle, ctypes.byref(motif(edges)), int(delta), int(c), float(p),
                                ctypes.byref(t), ctypes.byref(b), _stream(stream)), "tm_batch_config")
    return t.value, b.value


def batch_release(g: Graph, stream=None):
    """Drop the batched estimator's cached plans and stored anchor values of g."""
    _check(_lib.tm_batch_release(g.handle, _stream(stream)), "tm_batch_release")


class Server:
    """Continuous-batching query server over loaded graphs (see tm.h)."""

    def __init__(self, slots: int = 4, budget_bytes: int = 1 << 30):
        self._h = ctypes.c_void_p()
        _check(_lib.tm_server_create(int(slots), int(budget_bytes), ctypes.byref(self._h)), "tm_server_create")
        self._graphs = []

    def add_graph(self, g: Graph) -> int:
        gid = ctypes.c_int32()
        _check(_lib.tm_server_add_graph(self._h, g.handle, ctypes.byref(gid)), "tm_server_add_graph")
        self._graphs.append(g)
        return gid.value

    def submit(self, graph: int, edges, delta: int, kind: int = 0, c: int = 0, p: float = 0.0, seed: int = 0) -> int:
        q = Query(graph, kind, motif(edges), int(delta), int(c), float(p), int(seed))
        t = ctypes.c_int64()
        _check(_lib.tm_server_submit(self._h, ctypes.byref(q), ctypes.byref(t)), "tm_server_submit")
        return t.value

    def wait(self, ticket: int) -> dict:
        r = Result()
        _check(_lib.tm_server_wait(self._h, int(ticket), ctypes.byref(r)), "tm_server_wait")
        return {"status": r.status, "count": r.count.value(), "estimate": r.estimate, "latency_ms": r.latency_ms,
                "queue_ms": r.queue_ms, "batch_size": r.batch_size, "slot": r.slot, "ws_charged": r.ws_charged,
                "ws_measured": r.ws_measured}

    def stats(self) -> dict:
        s = ServerStats()
        _check(_lib.tm_server_stats_get(self._h, ctypes.byref(s)), "tm_server_stats_get")
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            _lib.tm_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return _lib.tm_version().decode()
