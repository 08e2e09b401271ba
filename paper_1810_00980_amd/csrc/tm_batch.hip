// Batched estimator: many independent estimates (one shift and one set of
// window draws per seed, Algorithm 1's outer loop over shifts run as
// separate estimators) of one three-edge motif in one persistent launch.
//
// Work is split into anchor tiles: runs of at most `tile` consecutive entries
// of one node's time-sorted incidence list.  The candidate tasks are the
// (tile, seed) pairs in tile-major order, so that at any moment the resident
// wavefronts work on the same region of the graph for every seed and share
// its cache lines.  Persistent wavefronts claim one tile's candidates (up to
// 64 seeds) at a time from one atomic counter (work stealing), keep those whose tile meets a window the
// seed keeps (one ballot), sweep each kept task's anchors that lie in kept
// windows, and add the motif's count and fixed-point weighted sum into that
// seed's accumulator.  A last kernel turns each seed's sum into its estimate.
// The kernels run as one hipGraph, captured once per (graph, motif, delta,
// c, p, seeds, tile, grid) and replayed with new seeds; counters are cleared
// by fill kernels, never by memset nodes.
//
// The tile size and the number of resident work-groups per CU are chosen by
// timing candidates on the first call (autotuner), per (graph, motif, delta,
// c, p).
//
// Stored anchor values: the weighted sum of the instances that start (or, for
// the stars swept backwards, end) at an anchor does not depend on the seed
// unless the anchor's delta-horizon crosses its window's edge.  When a batch
// covers at least one full pass over the anchors (seeds x p >= 1), one
// unclipped pass stores every anchor's count and weighted sum for the motif;
// the batch then adds the stored value of each anchor in a kept window whose
// horizon stays inside it and sweeps only the anchors within delta of the
// window's edge.  The sums are exact integers, so every seed's estimate is
// the same as the one the direct batch or a single call gives.
#include "tm_common.h"

#include <limits.h>
#include <string.h>

#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "tm_sweep_dev.h"

namespace {

using namespace sweepdev;

constexpr int BT_TPB = 256;

struct BatchArgs {
    int64_t n_seeds, J, L, delta;
    double p;
    const uint64_t *seeds;
    int64_t *shifts;          // [n_seeds]
    int32_t *kept_prefix;     // [n_seeds][J + 1]
    const int64_t *tiles;     // [n_tiles + 1] entry starts
    const int32_t *tile_node; // [n_tiles]
    int64_t n_tiles;
    unsigned long long *qctl; // [0] candidate counter
    uint64_t *out;            // [n_seeds][4]: count lo/hi, weight lo/hi
    const uint64_t *wfx;
    int32_t code;             // the motif's sweep code
    uint32_t want_fwd;
    int32_t want_bwd;
    double *z;                // [n_seeds]
    const uint64_t *vals;     // [entries][4] stored anchor values, or null
};

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// one work-group per seed: shift, and the prefix count of kept windows
__global__ void __launch_bounds__(BT_TPB) k_batch_flags(BatchArgs a) {
    __shared__ int32_t carry;
    __shared__ int32_t wsum[BT_TPB / TM_WAVE];
    int64_t k = blockIdx.x;
    uint64_t seed = a.seeds[k];
    if (threadIdx.x == 0) {
        uint32_t x0 = 0, x1 = 0, x2 = 0, x3 = 0;
        philox10_d(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
        uint64_t x = ((uint64_t)x1 << 32) | (uint64_t)x0;
        a.shifts[k] = -(int64_t)(x % (uint64_t)a.L);
        carry = 0;
        a.kept_prefix[k * (a.J + 1)] = 0;
    }
    __syncthreads();
    int lane = threadIdx.x & (TM_WAVE - 1), w = threadIdx.x / TM_WAVE;
    for (int64_t base = 1; base <= a.J; base += BT_TPB) {
        int64_t j = base + threadIdx.x;
        int32_t f = (j <= a.J && keep_window(seed, (uint64_t)j, a.p)) ? 1 : 0;
        // inclusive scan of f within the work-group
        int32_t v = f;
#pragma unroll
        for (int o = 1; o < TM_WAVE; o <<= 1) {
            int32_t y = __shfl_up(v, o, TM_WAVE);
            if (lane >= o) v += y;
        }
        if (lane == TM_WAVE - 1) wsum[w] = v;
        __syncthreads();
        int32_t add = carry;
        for (int i = 0; i < w; ++i) add += wsum[i];
        if (j <= a.J) a.kept_prefix[k * (a.J + 1) + j] = add + v;
        __syncthreads();
        if (threadIdx.x == BT_TPB - 1) carry = add + v;
        __syncthreads();
    }
}

__device__ inline void wave_sum_u128(uint64_t &lo, uint64_t &hi) {
#pragma unroll
    for (int o = TM_WAVE / 2; o > 0; o >>= 1) {
        uint64_t olo = __shfl_xor(lo, o, TM_WAVE);
        uint64_t ohi = __shfl_xor(hi, o, TM_WAVE);
        tm_add_u128(lo, hi, olo, ohi);
    }
}

// persistent wavefronts: claim (tile, seed) candidates, keep those whose
// tile meets a kept window of the seed, and for each kept task sweep the
// tile's anchors in kept windows with the lanes' own sums, reduce them across
// the wave and add them to the seed
template <int MODE, unsigned CLS>
__global__ void __launch_bounds__(BT_TPB) k_batch_sweep(DevGraph G, BatchArgs a) {
    const int lane = threadIdx.x & (TM_WAVE - 1);
    const int64_t total = a.n_tiles * a.n_seeds;
    // one claim covers one tile for up to 64 seeds
    const int64_t claim = a.n_seeds < TM_WAVE ? a.n_seeds : TM_WAVE;
    while (true) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd(&a.qctl[0], (unsigned long long)claim);
        base = __shfl(base, 0, TM_WAVE);
        if (base >= total) break;
        int64_t cand = base + lane;
        bool kept = false;
        if (lane < claim && cand < total) {
            int64_t t = cand / a.n_seeds, k = cand - t * a.n_seeds;
            int64_t s = a.shifts[k];
            int64_t e0 = a.tiles[t], e1 = a.tiles[t + 1];
            int64_t j0 = (G.inc_t[e0] - s) / a.L + 1, j1 = (G.inc_t[e1 - 1] - s) / a.L + 1;
            if (j1 > a.J) j1 = a.J;
            const int32_t *kp = a.kept_prefix + k * (a.J + 1);
            kept = kp[j1] - kp[j0 - 1] > 0;
        }
        unsigned long long todo = __ballot(kept);
        while (todo) {
            int b = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            int64_t id = base + b;
            int64_t t = id / a.n_seeds, k = id - t * a.n_seeds;
            int64_t e0 = a.tiles[t], e1 = a.tiles[t + 1];
            int64_t x = a.tile_node[t];
            int64_t lb = G.inc_off[x], le = G.inc_off[x + 1];
            SweepArgs sa;
            sa.delta = a.delta;
            sa.windowed = 1;
            sa.s = a.shifts[k];
            sa.L = a.L;
            sa.seed = a.seeds[k];
            sa.p = a.p;
            sa.wfx = a.wfx;
            sa.hist = nullptr;
            sa.out = nullptr;
            sa.counter = nullptr;
            sa.want_fwd = a.want_fwd;
            sa.n_entries = 0;
            sa.kidx = nullptr;
            sa.win = nullptr;
            OneCode one{a.code, 0, 0, 0, 0};
            for (int64_t i = e0 + lane; i < e1; i += TM_WAVE) {
                uint32_t nd = G.inc_nd[i];
                uint32_t y = nd & 0x7FFFFFFFu, d = nd >> 31;
                int64_t tt = G.inc_t[i];
                int64_t j = (tt - sa.s) / sa.L + 1;
                if (!keep_window(sa.seed, (uint64_t)j, sa.p)) continue;
                int64_t wlo = sa.s + (j - 1) * sa.L, whi = sa.s + j * sa.L - 1;
                if (a.vals && (CLS != 0u ? tt <= whi - a.delta : tt >= wlo + a.delta)) {
                    const uint64_t *v = a.vals + 4 * i;
                    tm_add_u128(one.cl, one.ch, v[0], v[1]);
                    tm_add_u128(one.wl, one.wh, v[2], v[3]);
                    continue;
                }
                if (CLS != 0u) {
                    int64_t hi = (tt > LLONG_MAX - a.delta) ? LLONG_MAX : tt + a.delta;
                    hi = hi < whi ? hi : whi;
                    sweep_fwd<MODE, CLS>(G, sa, i, le, y, d, tt, hi, wlo, nullptr, &one);
                } else {
                    int64_t lo = (tt < LLONG_MIN + a.delta) ? LLONG_MIN : tt - a.delta;
                    lo = lo > wlo ? lo : wlo;
                    sweep_bwd<MODE>(G, sa, i, lb, y, d, tt, lo, nullptr, &one);
                }
            }
            wave_sum_u128(one.cl, one.ch);
            wave_sum_u128(one.wl, one.wh);
            if (lane == 0) {
                uint64_t *o = a.out + 4 * k;
                if (one.cl | one.ch) tm_atomic_add_u128(o, o + 1, one.cl, one.ch);
                if (one.wl | one.wh) tm_atomic_add_u128(o + 2, o + 3, one.wl, one.wh);
            }
        }
    }
}

__global__ void k_batch_final(BatchArgs a) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_seeds) return;
    const uint64_t *o = a.out + 4 * k;
    double x = (double)o[3] * 18446744073709551616.0;
    x = x + (double)o[2];
    a.z[k] = x * (1.0 / 4503599627370496.0) / a.p;
}

// every anchor's unclipped count and weighted sum for one motif code
template <bool FWD, unsigned CLS>
__global__ void __launch_bounds__(BT_TPB) k_anchor_vals(DevGraph G, BatchArgs a, int64_t n_entries,
                                                         unsigned long long *counter, uint64_t *vals) {
    const int lane = threadIdx.x & (TM_WAVE - 1);
    SweepArgs sa;
    sa.delta = a.delta;
    sa.windowed = 0;
    sa.s = 0;
    sa.L = a.L;
    sa.seed = 0;
    sa.p = 1.0;
    sa.wfx = a.wfx;
    sa.hist = nullptr;
    sa.out = nullptr;
    sa.counter = nullptr;
    sa.want_fwd = a.want_fwd;
    sa.n_entries = 0;
    sa.kidx = nullptr;
    sa.win = nullptr;
    while (true) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd(counter, (unsigned long long)TM_WAVE);
        base = __shfl(base, 0, TM_WAVE);
        if (base >= n_entries) break;
        int64_t i = base + lane;
        if (i >= n_entries) continue;
        int64_t x = owner_of(G.inc_off, G.n, i);
        uint32_t nd = G.inc_nd[i];
        uint32_t y = nd & 0x7FFFFFFFu, d = nd >> 31;
        int64_t tt = G.inc_t[i];
        OneCode one{a.code, 0, 0, 0, 0};
        if (FWD) {
            int64_t hi = (tt > LLONG_MAX - a.delta) ? LLONG_MAX : tt + a.delta;
            sweep_fwd<MODE_WEIGHT, CLS>(G, sa, i, G.inc_off[x + 1], y, d, tt, hi, LLONG_MIN, nullptr, &one);
        } else {
            int64_t lo = (tt < LLONG_MIN + a.delta) ? LLONG_MIN : tt - a.delta;
            sweep_bwd<MODE_WEIGHT>(G, sa, i, G.inc_off[x], y, d, tt, lo, nullptr, &one);
        }
        uint64_t *v = vals + 4 * i;
        v[0] = one.cl;
        v[1] = one.ch;
        v[2] = one.wl;
        v[3] = one.wh;
    }
}

__global__ void k_weights_fx_b(int64_t delta, int64_t L, uint64_t *wfx) {
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d > delta) return;
    uint64_t den = (uint64_t)(L - d);
    uint64_t nhi = (uint64_t)L >> 12, nlo = (uint64_t)L << 52;
    uint64_t rem = nhi, q = 0;
    for (int b = 63; b >= 0; --b) {
        uint64_t top = rem >> 63;
        rem = (rem << 1) | ((nlo >> b) & 1ull);
        q <<= 1;
        if (top || rem >= den) {
            rem -= den;
            q |= 1ull;
        }
    }
    if (rem >= den - rem) q += 1;
    wfx[d] = q;
}

// node-aligned tiles of at most `tile` entries: tile starts and owners
__global__ void k_tile_count(const int64_t *inc_off, int64_t n, int64_t tile, int64_t *cnt) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    int64_t d = inc_off[x + 1] - inc_off[x];
    cnt[x] = (d + tile - 1) / tile;
}

__global__ void k_tile_fill(const int64_t *inc_off, int64_t n, int64_t tile, const int64_t *first, int64_t *tiles,
                            int32_t *tnode) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    int64_t b = inc_off[x], e = inc_off[x + 1];
    int64_t f = first[x];
    for (int64_t s = b, q = 0; s < e; s += tile, ++q) {
        tiles[f + q] = s;
        tnode[f + q] = (int32_t)x;
    }
}

__global__ void k_set_last(int64_t *tiles, int64_t n_tiles, int64_t v) { tiles[n_tiles] = v; }

// ------------------------------------------------------------------ host

struct BatchPlan {
    int64_t tile = 0, bpc = 0, n_seeds = 0, delta = 0, L = 0, J = 0, n_tiles = 0;
    int32_t code = -1;
    double p = 0;
    const uint64_t *vals = nullptr;  // stored anchor values (owned by the cache), or null
    DevBuf tiles, tnode, seeds, shifts, kp, qctl, out, wfx, z;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
    ~BatchPlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

using PlanKey = std::tuple<const tm_graph *, int32_t, int64_t, int64_t, double, int64_t, int64_t, int64_t>;
using TuneKey = std::tuple<const tm_graph *, int32_t, int64_t, int64_t, double>;
using ValKey = std::tuple<const tm_graph *, int32_t, int64_t, int64_t>;

struct BatchCache {
    std::mutex mu;
    std::map<PlanKey, std::unique_ptr<BatchPlan>> plans;
    std::map<TuneKey, std::pair<int64_t, int64_t>> tuned;
    std::map<ValKey, std::unique_ptr<DevBuf>> vals;  // stored anchor values per (graph, code, delta, L)
};
BatchCache &bcache() {
    static BatchCache c;
    return c;
}

BatchArgs make_args(BatchPlan &B, uint32_t want_fwd, int32_t want_bwd) {
    BatchArgs a;
    a.n_seeds = B.n_seeds;
    a.J = B.J;
    a.L = B.L;
    a.delta = B.delta;
    a.p = B.p;
    a.seeds = B.seeds.as<uint64_t>();
    a.shifts = B.shifts.as<int64_t>();
    a.kept_prefix = B.kp.as<int32_t>();
    a.tiles = B.tiles.as<int64_t>();
    a.tile_node = B.tnode.as<int32_t>();
    a.n_tiles = B.n_tiles;
    a.qctl = B.qctl.as<unsigned long long>();
    a.out = B.out.as<uint64_t>();
    a.wfx = B.wfx.as<uint64_t>();
    a.code = B.code;
    a.want_fwd = want_fwd;
    a.want_bwd = want_bwd;
    a.z = B.z.as<double>();
    a.vals = B.vals;
    return a;
}

uint32_t fwd_mask_of(int code) {
    if (code < 4) return 1;
    if (code < 12) return 2;
    if (code < 20) return 4;
    if (code < 28) return 8;
    return 0;
}

// the batch's kernel sequence on stream st (captured or not)
tm_status enqueue(const tm_graph *g, BatchPlan &B, hipStream_t st) {
    DevGraph G = dev_view(g);
    uint32_t wf = fwd_mask_of(B.code);
    int32_t wb = B.code >= 28 ? 1 : 0;
    BatchArgs a = make_args(B, wf, wb);
    int64_t nout = 4 * B.n_seeds;
    hipLaunchKernelGGL(k_fill_u64, dim3(tm_blocks(nout, 256)), dim3(256), 0, st, (unsigned long long *)a.out, nout,
                       0ull);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, a.qctl, (int64_t)2, 0ull);
    hipLaunchKernelGGL(k_batch_flags, dim3((unsigned)B.n_seeds), dim3(BT_TPB), 0, st, a);
    int dev = g->device, ncu = 0;
    TM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu <= 0) ncu = 256;
    unsigned nb = (unsigned)(ncu * B.bpc);
    switch (wf) {  // one kernel per sweep class, holding only that class's accumulators
        case 1: hipLaunchKernelGGL((k_batch_sweep<1, 1u>), dim3(nb), dim3(BT_TPB), 0, st, G, a); break;
        case 2: hipLaunchKernelGGL((k_batch_sweep<1, 2u>), dim3(nb), dim3(BT_TPB), 0, st, G, a); break;
        case 4: hipLaunchKernelGGL((k_batch_sweep<1, 4u>), dim3(nb), dim3(BT_TPB), 0, st, G, a); break;
        case 8: hipLaunchKernelGGL((k_batch_sweep<1, 8u>), dim3(nb), dim3(BT_TPB), 0, st, G, a); break;
        default: hipLaunchKernelGGL((k_batch_sweep<1, 0u>), dim3(nb), dim3(BT_TPB), 0, st, G, a); break;
    }
    hipLaunchKernelGGL(k_batch_final, dim3(tm_blocks(B.n_seeds, 64)), dim3(64), 0, st, a);
    return tm_hip_status(hipGetLastError());
}

tm_status build_plan(const tm_graph *g, BatchPlan &B, hipStream_t st) {
    int64_t n = g->n;
    // tiles
    DevBuf cnt, tot;
    TM_TRY(cnt.alloc((size_t)(n + 1) * 8));
    TM_TRY(tot.alloc(8));
    hipLaunchKernelGGL(k_tile_count, dim3(tm_blocks(n, 256)), dim3(256), 0, st, g->inc_off.as<int64_t>(), n, B.tile,
                       cnt.as<int64_t>());
    TM_HIP(hipGetLastError());
    TM_TRY(tm_scan_i64(cnt.as<int64_t>(), n, tot.as<int64_t>(), st));
    int64_t ntile = 0;
    TM_HIP(hipMemcpyAsync(&ntile, tot.p, 8, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    B.n_tiles = ntile;
    TM_TRY(B.tiles.alloc((size_t)(ntile + 1) * 8));
    TM_TRY(B.tnode.alloc((size_t)(ntile > 0 ? ntile : 1) * 4));
    hipLaunchKernelGGL(k_tile_fill, dim3(tm_blocks(n, 256)), dim3(256), 0, st, g->inc_off.as<int64_t>(), n, B.tile,
                       cnt.as<int64_t>(), B.tiles.as<int64_t>(), B.tnode.as<int32_t>());
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, st, B.tiles.as<int64_t>(), ntile, 2 * g->m_nl);
    TM_HIP(hipGetLastError());
    TM_TRY(B.seeds.alloc((size_t)B.n_seeds * 8));
    TM_TRY(B.shifts.alloc((size_t)B.n_seeds * 8));
    TM_TRY(B.kp.alloc((size_t)B.n_seeds * (B.J + 1) * 4));
    TM_TRY(B.qctl.alloc(64));
    TM_TRY(B.out.alloc((size_t)B.n_seeds * 32));
    TM_TRY(B.wfx.alloc((size_t)(B.delta + 1) * 8));
    TM_TRY(B.z.alloc((size_t)B.n_seeds * 8));
    hipLaunchKernelGGL(k_weights_fx_b, dim3(tm_blocks(B.delta + 1, 256)), dim3(256), 0, st, B.delta, B.L,
                       B.wfx.as<uint64_t>());
    TM_HIP(hipGetLastError());
    TM_HIP(hipStreamSynchronize(st));
    return TM_OK;
}

tm_status capture(const tm_graph *g, BatchPlan &B) {
    TM_HIP(hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    TM_HIP(hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal));
    tm_status s = enqueue(g, B, B.cap_stream);
    hipError_t e = hipStreamEndCapture(B.cap_stream, &graph);
    if (s != TM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    TM_HIP(e);
    e = hipGraphInstantiate(&B.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    TM_HIP(e);
    return TM_OK;
}

// Runs the batch (graph replay when captured) and copies the results.
tm_status run_plan(const tm_graph *g, BatchPlan &B, const uint64_t *seeds, double *est, tm_u128 *kept, bool use_graph,
                   hipStream_t st) {
    TM_HIP(hipMemcpyAsync(B.seeds.p, seeds, (size_t)B.n_seeds * 8, hipMemcpyHostToDevice, st));
    void *tok = tm_prof_begin(B.vals ? "count_batch_stored" : "count_batch", st);
    if (use_graph && B.exec) {
        TM_HIP(hipGraphLaunch(B.exec, st));
    } else {
        TM_TRY(enqueue(g, B, st));
    }
    tm_prof_end(tok, st);
    std::vector<double> z((size_t)B.n_seeds);
    std::vector<uint64_t> o((size_t)B.n_seeds * 4);
    TM_HIP(hipMemcpyAsync(z.data(), B.z.p, (size_t)B.n_seeds * 8, hipMemcpyDeviceToHost, st));
    TM_HIP(hipMemcpyAsync(o.data(), B.out.p, (size_t)B.n_seeds * 32, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    for (int64_t k = 0; k < B.n_seeds; ++k) {
        if (est) est[k] = z[(size_t)k];
        if (kept) {
            kept[k].lo = o[(size_t)(4 * k)];
            kept[k].hi = o[(size_t)(4 * k + 1)];
        }
    }
    return TM_OK;
}

// Stored anchor values of (graph, code, delta, L) for plan B, computed on
// first use with B's weights; *vals stays null when they do not fit in a
// quarter of the free device memory.
tm_status anchor_vals(const tm_graph *g, BatchPlan &B, const uint64_t **vals, hipStream_t st) {
    BatchCache &C = bcache();
    ValKey key{g, B.code, B.delta, B.L};
    {
        std::lock_guard<std::mutex> lk(C.mu);
        auto it = C.vals.find(key);
        if (it != C.vals.end()) {
            *vals = it->second->as<uint64_t>();
            return TM_OK;
        }
    }
    *vals = nullptr;
    int64_t ne = 2 * g->m_nl;
    size_t bytes = (size_t)ne * 32;
    size_t fr = 0, tot = 0;
    TM_HIP(hipMemGetInfo(&fr, &tot));
    if (bytes > fr / 4) return TM_OK;
    std::unique_ptr<DevBuf> V(new (std::nothrow) DevBuf());
    if (!V) return TM_ENOMEM;
    TM_TRY(V->alloc(bytes));
    DevBuf ctr;
    TM_TRY(ctr.alloc(64));
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, ctr.as<unsigned long long>(), (int64_t)1, 0ull);
    DevGraph G = dev_view(g);
    BatchArgs a = make_args(B, fwd_mask_of(B.code), B.code >= 28 ? 1 : 0);
    int dev = g->device, ncu = 0;
    TM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu <= 0) ncu = 256;
    void *tok = tm_prof_begin("batch_anchor_values", st);
    dim3 grid((unsigned)(ncu * 8)), blk(BT_TPB);
    unsigned long long *cp = ctr.as<unsigned long long>();
    uint64_t *vp = V->as<uint64_t>();
    switch (a.want_bwd ? 0u : a.want_fwd) {
        case 1: hipLaunchKernelGGL((k_anchor_vals<true, 1u>), grid, blk, 0, st, G, a, ne, cp, vp); break;
        case 2: hipLaunchKernelGGL((k_anchor_vals<true, 2u>), grid, blk, 0, st, G, a, ne, cp, vp); break;
        case 4: hipLaunchKernelGGL((k_anchor_vals<true, 4u>), grid, blk, 0, st, G, a, ne, cp, vp); break;
        case 8: hipLaunchKernelGGL((k_anchor_vals<true, 8u>), grid, blk, 0, st, G, a, ne, cp, vp); break;
        default: hipLaunchKernelGGL((k_anchor_vals<false, 0u>), grid, blk, 0, st, G, a, ne, cp, vp); break;
    }
    TM_HIP(hipGetLastError());
    tm_prof_end(tok, st);
    TM_HIP(hipStreamSynchronize(st));
    std::lock_guard<std::mutex> lk(C.mu);
    auto it = C.vals.find(key);
    if (it == C.vals.end()) it = C.vals.emplace(key, std::move(V)).first;
    *vals = it->second->as<uint64_t>();
    return TM_OK;
}

tm_status get_plan(const tm_graph *g, int32_t code, int64_t delta, int64_t L, double p, int64_t n_seeds, int64_t tile,
                   int64_t bpc, bool want_graph, BatchPlan **out, hipStream_t st) {
    BatchCache &C = bcache();
    PlanKey key{g, code, delta, L, p, n_seeds, tile, bpc};
    {
        std::lock_guard<std::mutex> lk(C.mu);
        auto it = C.plans.find(key);
        if (it != C.plans.end()) {
            *out = it->second.get();
            return TM_OK;
        }
    }
    std::unique_ptr<BatchPlan> B(new (std::nothrow) BatchPlan());
    if (!B) return TM_ENOMEM;
    B->tile = tile;
    B->bpc = bpc;
    B->n_seeds = n_seeds;
    B->delta = delta;
    B->L = L;
    B->p = p;
    B->code = code;
    B->J = 1 + g->t_span / L + ((g->t_span % L) ? 1 : 0);
    TM_TRY(build_plan(g, *B, st));
    if ((double)n_seeds * p >= 1.0) TM_TRY(anchor_vals(g, *B, &B->vals, st));
    if (want_graph) TM_TRY(capture(g, *B));
    std::lock_guard<std::mutex> lk(C.mu);
    BatchPlan *raw = B.get();
    C.plans[key] = std::move(B);
    *out = raw;
    return TM_OK;
}

}  // namespace

// Drop every cached batch plan of graph g (called when it is freed).
void tm_batch_forget(const tm_graph *g) {
    BatchCache &C = bcache();
    std::lock_guard<std::mutex> lk(C.mu);
    for (auto it = C.plans.begin(); it != C.plans.end();) {
        if (std::get<0>(it->first) == g) it = C.plans.erase(it);
        else ++it;
    }
    for (auto it = C.tuned.begin(); it != C.tuned.end();) {
        if (std::get<0>(it->first) == g) it = C.tuned.erase(it);
        else ++it;
    }
    for (auto it = C.vals.begin(); it != C.vals.end();) {
        if (std::get<0>(it->first) == g) it = C.vals.erase(it);
        else ++it;
    }
}

// Drop the cached batch plans and stored anchor values of graph g, keeping
// its tuning results (the caller reclaims device memory, or times a cold run).
void tm_batch_release_plans(const tm_graph *g) {
    BatchCache &C = bcache();
    std::lock_guard<std::mutex> lk(C.mu);
    for (auto it = C.plans.begin(); it != C.plans.end();) {
        if (std::get<0>(it->first) == g) it = C.plans.erase(it);
        else ++it;
    }
    for (auto it = C.vals.begin(); it != C.vals.end();) {
        if (std::get<0>(it->first) == g) it = C.vals.erase(it);
        else ++it;
    }
}

// Autotuner: times the uncaptured batch on up to 8 seeds for each candidate
// (tile, work-groups per CU) and keeps the fastest.
tm_status tm_batch_tune(const tm_graph *g, int32_t code, int64_t delta, int64_t L, double p, int64_t *tile,
                        int64_t *bpc, hipStream_t st) {
    BatchCache &C = bcache();
    TuneKey key{g, code, delta, L, p};
    {
        std::lock_guard<std::mutex> lk(C.mu);
        auto it = C.tuned.find(key);
        if (it != C.tuned.end()) {
            *tile = it->second.first;
            *bpc = it->second.second;
            return TM_OK;
        }
    }
    const int64_t tiles[] = {64, 256, 1024};
    const int64_t bpcs[] = {8, 16};
    const int64_t NS = 2;
    uint64_t seeds[NS];
    for (int i = 0; i < NS; ++i) seeds[i] = 0x5EED0000ull + (uint64_t)i;
    double best = 1e300;
    int64_t bt = 1024, bb = 4;
    hipEvent_t e0, e1;
    TM_HIP(hipEventCreate(&e0));
    TM_HIP(hipEventCreate(&e1));
    for (int64_t t : tiles) {
        for (int64_t b : bpcs) {
            BatchPlan *B = nullptr;
            tm_status s = get_plan(g, code, delta, L, p, NS, t, b, false, &B, st);
            if (s != TM_OK) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return s;
            }
            (void)hipMemcpyAsync(B->seeds.p, seeds, sizeof seeds, hipMemcpyHostToDevice, st);
            (void)hipEventRecord(e0, st);
            (void)enqueue(g, *B, st);
            (void)hipEventRecord(e1, st);
            (void)hipStreamSynchronize(st);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) {
                best = ms;
                bt = t;
                bb = b;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        // tuning plans (8 seeds, uncaptured) are not needed any more
        std::lock_guard<std::mutex> lk(C.mu);
        for (auto it = C.plans.begin(); it != C.plans.end();) {
            if (std::get<0>(it->first) == g && std::get<5>(it->first) == 2 && !it->second->exec)
                it = C.plans.erase(it);
            else
                ++it;
        }
        C.tuned[key] = {bt, bb};
    }
    *tile = bt;
    *bpc = bb;
    return TM_OK;
}

tm_status tm_batch_run(const tm_graph *g, int32_t code, int64_t delta, int64_t L, double p, int64_t n_seeds,
                       const uint64_t *seeds, int64_t tile, int64_t bpc, double *est, tm_u128 *kept,
                       hipStream_t st) {
    if (n_seeds <= 0) return TM_OK;
    if (g->m_nl == 0) {
        for (int64_t k = 0; k < n_seeds; ++k) {
            if (est) est[k] = 0.0;
            if (kept) kept[k].lo = kept[k].hi = 0;
        }
        return TM_OK;
    }
    BatchPlan *B = nullptr;
    TM_TRY(get_plan(g, code, delta, L, p, n_seeds, tile, bpc, true, &B, st));
    return run_plan(g, *B, seeds, est, kept, true, st);
}
