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
    const uint64_t *vals = nullptr;  // stored anchor values, or null
    std::shared_ptr<DevBuf> vals_buf; // keeps them alive while the plan lives
    DevBuf tiles, tnode, seeds, shifts, kp, qctl, out, wfx, z;
    // One run at a time: a run writes the plan's seeds, queue counters and
    // outputs and replays its one hipGraphExec.  Concurrent callers with the
    // same key (other threads, other streams) wait here.
    std::mutex run_mu;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
    ~BatchPlan() {
        std::shared_lock<std::shared_mutex> lk(tm_capture_lock());  // may synchronise
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

using PlanKey = std::tuple<const tm_graph *, int32_t, int64_t, int64_t, double, int64_t, int64_t, int64_t>;
using TuneKey = std::tuple<const tm_graph *, int32_t, int64_t, int64_t, double>;
using ValKey = std::tuple<const tm_graph *, int32_t, int64_t, int64_t>;

// Plans and stored values are shared: dropping them from the cache (release,
// tuning clean-up) leaves a plan that another thread is running alive until
// that run ends.
struct BatchCache {
    std::mutex mu;
    std::map<PlanKey, std::shared_ptr<BatchPlan>> plans;
    std::map<TuneKey, std::pair<int64_t, int64_t>> tuned;
    std::map<ValKey, std::shared_ptr<DevBuf>> vals;  // stored anchor values per (graph, code, delta, L)
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
    TM_HIP(tm_locked_call([&] { return hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking); }));
    hipGraph_t graph = nullptr;
    tm_status s;
    hipError_t e;
    {
        // no library free (an implicit device synchronisation) during the capture
        std::unique_lock<std::shared_mutex> lk(tm_capture_lock());
        e = hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return tm_hip_status(e);
        s = enqueue(g, B, B.cap_stream);
        e = hipStreamEndCapture(B.cap_stream, &graph);
    }
    if (s != TM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    TM_HIP(e);
    e = tm_locked_call([&] { return hipGraphInstantiate(&B.exec, graph, nullptr, nullptr, 0); });
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
tm_status anchor_vals(const tm_graph *g, BatchPlan &B, std::shared_ptr<DevBuf> *vals, hipStream_t st) {
    BatchCache &C = bcache();
    ValKey key{g, B.code, B.delta, B.L};
    {
        std::lock_guard<std::mutex> lk(C.mu);
        auto it = C.vals.find(key);
        if (it != C.vals.end()) {
            *vals = it->second;
            return TM_OK;
        }
    }
    vals->reset();
    int64_t ne = 2 * g->m_nl;
    size_t bytes = (size_t)ne * 32;
    size_t fr = 0, tot = 0;
    TM_HIP(hipMemGetInfo(&fr, &tot));
    if (bytes > fr / 4) return TM_OK;
    std::shared_ptr<DevBuf> V(new (std::nothrow) DevBuf());
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
    // a thread that computed the same values first wins; ours are dropped
    *vals = C.vals.try_emplace(key, std::move(V)).first->second;
    return TM_OK;
}

tm_status get_plan(const tm_graph *g, int32_t code, int64_t delta, int64_t L, double p, int64_t n_seeds, int64_t tile,
                   int64_t bpc, bool want_graph, std::shared_ptr<BatchPlan> *out, hipStream_t st) {
    BatchCache &C = bcache();
    PlanKey key{g, code, delta, L, p, n_seeds, tile, bpc};
    {
        std::lock_guard<std::mutex> lk(C.mu);
        auto it = C.plans.find(key);
        if (it != C.plans.end()) {
            *out = it->second;
            return TM_OK;
        }
    }
    std::shared_ptr<BatchPlan> B(new (std::nothrow) BatchPlan());
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
    if ((double)n_seeds * p >= 1.0) {
        TM_TRY(anchor_vals(g, *B, &B->vals_buf, st));
        B->vals = B->vals_buf ? B->vals_buf->as<uint64_t>() : nullptr;
    }
    if (want_graph) TM_TRY(capture(g, *B));
    std::lock_guard<std::mutex> lk(C.mu);
    // a thread that built the same plan first wins; ours is dropped unused
    *out = C.plans.try_emplace(key, std::move(B)).first->second;
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
    TM_HIP(tm_locked_call([&] { return hipEventCreate(&e0); }));
    TM_HIP(tm_locked_call([&] { return hipEventCreate(&e1); }));
    for (int64_t t : tiles) {
        for (int64_t b : bpcs) {
            std::shared_ptr<BatchPlan> B;
            tm_status s = get_plan(g, code, delta, L, p, NS, t, b, false, &B, st);
            if (s != TM_OK) {
                (void)tm_locked_call([&] { return hipEventDestroy(e0); });
                (void)tm_locked_call([&] { return hipEventDestroy(e1); });
                return s;
            }
            std::lock_guard<std::mutex> run(B->run_mu);
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
    (void)tm_locked_call([&] { return hipEventDestroy(e0); });
    (void)tm_locked_call([&] { return hipEventDestroy(e1); });
    {
        // tuning plans (2 seeds, uncaptured) are not needed any more; one
        // that another thread is running stays alive until its run ends
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
    std::shared_ptr<BatchPlan> B;
    TM_TRY(get_plan(g, code, delta, L, p, n_seeds, tile, bpc, true, &B, st));
    std::lock_guard<std::mutex> run(B->run_mu);
    return run_plan(g, *B, seeds, est, kept, true, st);
}

// ---------------------------------------------------------- mixed batches
//
// Estimates of many queries on one graph in one captured launch: each
// estimator has its own three-edge motif, delta, window length c delta,
// sampling probability and seed (Algorithm 1 run once per query, the loop
// over its windows in parallel, all queries' windows together).  The
// candidate tasks are (tile, estimator) pairs, tile-major, so that waves
// working on one region of the graph serve every estimator that keeps it.
// Each sweep class has a kernel of its own, holding only that class's
// accumulators, over the estimators of that class; the kernels run as
// parallel branches of one hipGraph and steal work from their own queues.
// Sums are exact integers, so every estimate equals what a single call gives.

namespace {

// one estimator of a mixed batch
struct MixEst {
    int64_t delta, L, J;
    int64_t s;       // shift (k_mix_flags)
    int64_t kp_off;  // its kept-window prefix: kp[kp_off .. kp_off + J]
    int64_t w_off;   // its weights: wfx[w_off .. w_off + delta]
    double p;
    uint64_t seed;
    int32_t code;
    uint32_t want_fwd;  // 1, 2, 4, 8: forward class; 0: backward stars
};

struct MixArgs {
    const MixEst *est;       // [n_est]
    const int32_t *cls_est;  // estimators of this kernel's class
    int64_t n_cls;
    int32_t *kp;
    const uint64_t *wfx;
    const int64_t *tiles;
    const int32_t *tile_node;
    int64_t n_tiles;
    unsigned long long *qctl;  // this class's candidate counter
    uint64_t *out;             // [n_est][4]
};

// one work-group per estimator: its shift and the prefix count of its kept windows
__global__ void __launch_bounds__(BT_TPB) k_mix_flags(MixEst *E, int32_t *kp) {
    __shared__ int32_t carry;
    __shared__ int32_t wsum[BT_TPB / TM_WAVE];
    MixEst &e = E[blockIdx.x];
    const uint64_t seed = e.seed;
    const int64_t J = e.J;
    int32_t *pre = kp + e.kp_off;
    if (threadIdx.x == 0) {
        uint32_t x0 = 0, x1 = 0, x2 = 0, x3 = 0;
        philox10_d(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
        const uint64_t x = ((uint64_t)x1 << 32) | (uint64_t)x0;
        e.s = -(int64_t)(x % (uint64_t)e.L);
        carry = 0;
        pre[0] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & (TM_WAVE - 1), w = threadIdx.x / TM_WAVE;
    for (int64_t base = 1; base <= J; base += BT_TPB) {
        const int64_t j = base + threadIdx.x;
        const int32_t f = (j <= J && keep_window(seed, (uint64_t)j, e.p)) ? 1 : 0;
        int32_t v = f;
#pragma unroll
        for (int o = 1; o < TM_WAVE; o <<= 1) {
            const int32_t y = __shfl_up(v, o, TM_WAVE);
            if (lane >= o) v += y;
        }
        if (lane == TM_WAVE - 1) wsum[w] = v;
        __syncthreads();
        int32_t add = carry;
        for (int i = 0; i < w; ++i) add += wsum[i];
        if (j <= J) pre[j] = add + v;
        __syncthreads();
        if (threadIdx.x == BT_TPB - 1) carry = add + v;
        __syncthreads();
    }
}

// weights round(2^52 L / (L - d)) of every estimator (grid y = estimator)
__global__ void k_mix_weights(const MixEst *E, uint64_t *wfx) {
    const MixEst &e = E[blockIdx.y];
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d <= e.delta; d += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t den = (uint64_t)(e.L - d);
        const uint64_t nhi = (uint64_t)e.L >> 12, nlo = (uint64_t)e.L << 52;
        uint64_t rem = nhi, q = 0;
        for (int b = 63; b >= 0; --b) {
            const uint64_t top = rem >> 63;
            rem = (rem << 1) | ((nlo >> b) & 1ull);
            q <<= 1;
            if (top || rem >= den) {
                rem -= den;
                q |= 1ull;
            }
        }
        if (rem >= den - rem) q += 1;
        wfx[e.w_off + d] = q;
    }
}

// persistent waves of one sweep class: claim (tile, estimator) candidates,
// keep those whose tile meets a window the estimator keeps (one ballot), and
// sweep each kept task's anchors in kept windows with that estimator's delta,
// windows and weights
template <unsigned CLS>
__global__ void __launch_bounds__(BT_TPB) k_mix_sweep(DevGraph G, MixArgs a) {
    const int lane = threadIdx.x & (TM_WAVE - 1);
    const int64_t total = a.n_tiles * a.n_cls;
    const int64_t claim = a.n_cls < TM_WAVE ? a.n_cls : TM_WAVE;
    while (true) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd(a.qctl, (unsigned long long)claim);
        base = __shfl(base, 0, TM_WAVE);
        if (base >= total) break;
        const int64_t cand = base + lane;
        bool kept = false;
        if (lane < claim && cand < total) {
            const int64_t t = cand / a.n_cls, k = a.cls_est[cand - t * a.n_cls];
            const MixEst &e = a.est[k];
            const int64_t e0 = a.tiles[t], e1 = a.tiles[t + 1];
            const int64_t j0 = (G.inc_t[e0] - e.s) / e.L + 1;
            int64_t j1 = (G.inc_t[e1 - 1] - e.s) / e.L + 1;
            if (j1 > e.J) j1 = e.J;
            const int32_t *kp = a.kp + e.kp_off;
            kept = kp[j1] - kp[j0 - 1] > 0;
        }
        unsigned long long todo = __ballot(kept);
        while (todo) {
            const int b = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const int64_t id = base + b;
            const int64_t t = id / a.n_cls, k = a.cls_est[id - t * a.n_cls];
            const MixEst e = a.est[k];
            const int64_t e0 = a.tiles[t], e1 = a.tiles[t + 1];
            const int64_t x = a.tile_node[t];
            const int64_t lb = G.inc_off[x], le = G.inc_off[x + 1];
            SweepArgs sa;
            sa.delta = e.delta;
            sa.windowed = 1;
            sa.s = e.s;
            sa.L = e.L;
            sa.seed = e.seed;
            sa.p = e.p;
            sa.wfx = a.wfx + e.w_off;
            sa.hist = nullptr;
            sa.out = nullptr;
            sa.counter = nullptr;
            sa.want_fwd = CLS;
            sa.n_entries = 0;
            sa.kidx = nullptr;
            sa.win = nullptr;
            OneCode one{e.code, 0, 0, 0, 0};
            for (int64_t i = e0 + lane; i < e1; i += TM_WAVE) {
                const uint32_t nd = G.inc_nd[i];
                const uint32_t y = nd & 0x7FFFFFFFu, d = nd >> 31;
                const int64_t tt = G.inc_t[i];
                const int64_t j = (tt - sa.s) / sa.L + 1;
                if (!keep_window(sa.seed, (uint64_t)j, sa.p)) continue;
                const int64_t wlo = sa.s + (j - 1) * sa.L, whi = sa.s + j * sa.L - 1;
                if (CLS != 0u) {
                    int64_t hi = (tt > LLONG_MAX - e.delta) ? LLONG_MAX : tt + e.delta;
                    hi = hi < whi ? hi : whi;
                    sweep_fwd<MODE_WEIGHT, CLS>(G, sa, i, le, y, d, tt, hi, wlo, nullptr, &one);
                } else {
                    int64_t lo = (tt < LLONG_MIN + e.delta) ? LLONG_MIN : tt - e.delta;
                    lo = lo > wlo ? lo : wlo;
                    sweep_bwd<MODE_WEIGHT>(G, sa, i, lb, y, d, tt, lo, nullptr, &one);
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

__global__ void k_mix_final(const MixEst *E, const uint64_t *out, int64_t n, double *z) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint64_t *o = out + 4 * k;
    double x = (double)o[3] * 18446744073709551616.0;
    x = x + (double)o[2];
    z[k] = x * (1.0 / 4503599627370496.0) / E[k].p;
}

constexpr int MIX_CLASSES = 5;
const uint32_t kMixClass[MIX_CLASSES] = {1u, 2u, 4u, 8u, 0u};

int mix_class_index(int code) {
    if (code < 4) return 0;
    if (code < 12) return 1;
    if (code < 20) return 2;
    if (code < 28) return 3;
    return 4;
}

// A mixed batch's device buffers, per host thread and grow-only (a free is a
// device-wide synchronisation, which would stall the other threads' work),
// their sizes bounded by mix_bytes.
struct MixBufs {
    DevBuf est, cls_est, kp, wfx, tiles, tnode, qctl, out, z, cnt, tot;
};
thread_local MixBufs t_mix;

struct MixPlan {
    int64_t n = 0, tile = 0, bpc = 0, n_tiles = 0, kp_words = 0, w_words = 0;
    int64_t n_cls[MIX_CLASSES] = {0, 0, 0, 0, 0}, cls_off[MIX_CLASSES] = {0, 0, 0, 0, 0};
    MixBufs &b = t_mix;
    DevBuf &est = b.est, &cls_est = b.cls_est, &kp = b.kp, &wfx = b.wfx, &tiles = b.tiles, &tnode = b.tnode,
           &qctl = b.qctl, &out = b.out, &z = b.z, &cnt = b.cnt, &tot = b.tot;
    hipStream_t *side = nullptr;
    hipEvent_t fork = nullptr, *join = nullptr;
    hipGraphExec_t exec = nullptr;
    ~MixPlan() {
        if (exec) {
            std::shared_lock<std::shared_mutex> lk(tm_capture_lock());  // may synchronise
            (void)hipGraphExecDestroy(exec);
        }
    }
};

// Per host thread: the capture stream, the class branches' streams (default
// priority) and their fork/join events, created on first use and kept until
// the process ends (destroying them at thread exit could run after the
// runtime's teardown).
struct MixStreams {
    bool ok = false;
    hipStream_t cap = nullptr, side[MIX_CLASSES] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[MIX_CLASSES] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

MixStreams *mix_streams() {
    thread_local MixStreams S;
    if (!S.ok) {
        std::shared_lock<std::shared_mutex> lk(tm_capture_lock());
        bool ok = hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&S.fork, hipEventDisableTiming) == hipSuccess;
        for (int c = 0; c < MIX_CLASSES; ++c) {
            ok = ok && hipStreamCreateWithFlags(&S.side[c], hipStreamNonBlocking) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&S.join[c], hipEventDisableTiming) == hipSuccess;
        }
        if (!ok) {
            (void)hipGetLastError();
            return nullptr;
        }
        S.ok = true;
    }
    return &S;
}

// device bytes of every buffer a mixed batch allocates (DevBuf sizes)
int64_t mix_bytes(const tm_graph *g, int64_t n, const int64_t *delta, const int64_t *L, int64_t tile,
                  int64_t *n_tiles_ub, int64_t *kp_words, int64_t *w_words) {
    int64_t kw = 0, ww = 0;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t J = 1 + g->t_span / L[k] + ((g->t_span % L[k]) ? 1 : 0);
        kw += J + 1;
        ww += delta[k] + 1;
    }
    // node-aligned tiles: at most one partial tile per node plus full ones
    const int64_t nt = (2 * g->m_nl) / tile + g->n + 1;
    if (n_tiles_ub) *n_tiles_ub = nt;
    if (kp_words) *kp_words = kw;
    if (w_words) *w_words = ww;
    const int64_t n1 = n > 0 ? n : 1;
    return (int64_t)sizeof(MixEst) * n1 + 4 * n1 + 4 * kw + 8 * ww + 8 * (nt + 1) + 4 * nt + 64 + 32 * n1 +
           8 * n1 + 8 * (g->n + 1) + 8;
}

tm_status mix_enqueue(const tm_graph *g, MixPlan &B, hipStream_t st, bool fork_streams) {
    DevGraph G = dev_view(g);
    MixEst *E = B.est.as<MixEst>();
    hipLaunchKernelGGL(k_fill_u64, dim3(tm_blocks(4 * B.n, 256)), dim3(256), 0, st, (unsigned long long *)B.out.p,
                       4 * B.n, 0ull);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, B.qctl.as<unsigned long long>(), (int64_t)8, 0ull);
    hipLaunchKernelGGL(k_mix_flags, dim3((unsigned)B.n), dim3(BT_TPB), 0, st, E, B.kp.as<int32_t>());
    TM_HIP(hipGetLastError());
    int dev = g->device, ncu = 0;
    TM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu <= 0) ncu = 256;
    int used = 0;
    for (int c = 0; c < MIX_CLASSES; ++c) used += B.n_cls[c] > 0;
    if (fork_streams && used > 1) TM_HIP(hipEventRecord(B.fork, st));
    int branch = 0;
    for (int c = 0; c < MIX_CLASSES; ++c) {
        if (!B.n_cls[c]) continue;
        hipStream_t sk = st;
        if (fork_streams && used > 1 && branch++ > 0) {
            sk = B.side[c];
            TM_HIP(hipStreamWaitEvent(sk, B.fork, 0));
        }
        MixArgs a;
        a.est = E;
        a.cls_est = B.cls_est.as<int32_t>() + B.cls_off[c];
        a.n_cls = B.n_cls[c];
        a.kp = B.kp.as<int32_t>();
        a.wfx = B.wfx.as<uint64_t>();
        a.tiles = B.tiles.as<int64_t>();
        a.tile_node = B.tnode.as<int32_t>();
        a.n_tiles = B.n_tiles;
        a.qctl = B.qctl.as<unsigned long long>() + c;
        a.out = B.out.as<uint64_t>();
        const unsigned nb = (unsigned)(ncu * B.bpc);
        switch (kMixClass[c]) {
            case 1u: hipLaunchKernelGGL((k_mix_sweep<1u>), dim3(nb), dim3(BT_TPB), 0, sk, G, a); break;
            case 2u: hipLaunchKernelGGL((k_mix_sweep<2u>), dim3(nb), dim3(BT_TPB), 0, sk, G, a); break;
            case 4u: hipLaunchKernelGGL((k_mix_sweep<4u>), dim3(nb), dim3(BT_TPB), 0, sk, G, a); break;
            case 8u: hipLaunchKernelGGL((k_mix_sweep<8u>), dim3(nb), dim3(BT_TPB), 0, sk, G, a); break;
            default: hipLaunchKernelGGL((k_mix_sweep<0u>), dim3(nb), dim3(BT_TPB), 0, sk, G, a); break;
        }
        TM_HIP(hipGetLastError());
        if (sk != st) {
            TM_HIP(hipEventRecord(B.join[c], sk));
            TM_HIP(hipStreamWaitEvent(st, B.join[c], 0));
        }
    }
    hipLaunchKernelGGL(k_mix_final, dim3(tm_blocks(B.n, 64)), dim3(64), 0, st, (const MixEst *)E,
                       (const uint64_t *)B.out.p, B.n, B.z.as<double>());
    return tm_hip_status(hipGetLastError());
}

}  // namespace

// Estimates of n three-edge-motif queries (sweep codes) on graph g in one
// captured launch; each query has its own delta, window length L, p and
// seed.  ws_bytes (nullable) receives the device bytes the batch allocated.
tm_status tm_batch_mixed(const tm_graph *g, int64_t n, const int32_t *code, const int64_t *delta, const int64_t *L,
                         const double *p, const uint64_t *seeds, double *est, tm_u128 *kept, hipStream_t st,
                         bool capture) {
    if (n <= 0) return TM_OK;
    if (g->m_nl == 0) {
        for (int64_t k = 0; k < n; ++k) {
            est[k] = 0.0;
            if (kept) kept[k].lo = kept[k].hi = 0;
        }
        return TM_OK;
    }
    MixPlan B;
    B.n = n;
    B.tile = 256;
    B.bpc = 8;
    int64_t nt_ub = 0;
    mix_bytes(g, n, delta, L, B.tile, &nt_ub, &B.kp_words, &B.w_words);
    // estimators, grouped by sweep class
    std::vector<MixEst> E((size_t)n);
    std::vector<int32_t> order;
    order.reserve((size_t)n);
    int64_t kw = 0, ww = 0;
    for (int64_t k = 0; k < n; ++k) {
        MixEst &e = E[(size_t)k];
        e.delta = delta[k];
        e.L = L[k];
        e.J = 1 + g->t_span / L[k] + ((g->t_span % L[k]) ? 1 : 0);
        e.s = 0;
        e.kp_off = kw;
        e.w_off = ww;
        e.p = p[k];
        e.seed = seeds[k];
        e.code = code[k];
        const int c = mix_class_index(code[k]);
        e.want_fwd = kMixClass[c];
        kw += e.J + 1;
        ww += e.delta + 1;
        B.n_cls[c] += 1;
    }
    for (int c = 0, off = 0; c < MIX_CLASSES; ++c) {
        B.cls_off[c] = off;
        off += (int)B.n_cls[c];
        for (int64_t k = 0; k < n; ++k)
            if (mix_class_index(code[k]) == c) order.push_back((int32_t)k);
    }
    TM_TRY(B.est.reserve((size_t)n * sizeof(MixEst)));
    TM_TRY(B.cls_est.reserve((size_t)n * 4));
    TM_TRY(B.kp.reserve((size_t)kw * 4));
    TM_TRY(B.wfx.reserve((size_t)ww * 8));
    TM_TRY(B.qctl.reserve(64));
    TM_TRY(B.out.reserve((size_t)n * 32));
    TM_TRY(B.z.reserve((size_t)n * 8));
    TM_HIP(hipMemcpyAsync(B.est.p, E.data(), (size_t)n * sizeof(MixEst), hipMemcpyHostToDevice, st));
    TM_HIP(hipMemcpyAsync(B.cls_est.p, order.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
    // node-aligned tiles of at most B.tile entries
    const int64_t nn = g->n;
    TM_TRY(B.cnt.reserve((size_t)(nn + 1) * 8));
    TM_TRY(B.tot.reserve(8));
    hipLaunchKernelGGL(k_tile_count, dim3(tm_blocks(nn, 256)), dim3(256), 0, st, g->inc_off.as<int64_t>(), nn, B.tile,
                       B.cnt.as<int64_t>());
    TM_HIP(hipGetLastError());
    TM_TRY(tm_scan_i64(B.cnt.as<int64_t>(), nn, B.tot.as<int64_t>(), st));
    int64_t ntile = 0;
    TM_HIP(hipMemcpyAsync(&ntile, B.tot.p, 8, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    if (ntile > nt_ub) return TM_EDEVICE;  // the bound mix_bytes charges
    B.n_tiles = ntile;
    TM_TRY(B.tiles.reserve((size_t)(nt_ub + 1) * 8));
    TM_TRY(B.tnode.reserve((size_t)nt_ub * 4));
    hipLaunchKernelGGL(k_tile_fill, dim3(tm_blocks(nn, 256)), dim3(256), 0, st, g->inc_off.as<int64_t>(), nn, B.tile,
                       B.cnt.as<int64_t>(), B.tiles.as<int64_t>(), B.tnode.as<int32_t>());
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, st, B.tiles.as<int64_t>(), ntile, 2 * g->m_nl);
    int64_t maxd = 0;
    for (int64_t k = 0; k < n; ++k) maxd = std::max<int64_t>(maxd, delta[k]);
    unsigned gx = tm_blocks(maxd + 1, 256);
    if (gx > 1024) gx = 1024;
    hipLaunchKernelGGL(k_mix_weights, dim3(gx, (unsigned)n), dim3(256), 0, st, (const MixEst *)B.est.as<MixEst>(),
                       B.wfx.as<uint64_t>());
    TM_HIP(hipGetLastError());
    // the launch sequence (the class kernels as parallel branches): captured
    // on this thread's capture stream and replayed on the caller's stream, or
    // enqueued on the caller's stream with the same fork and join
    MixStreams *MS = mix_streams();
    if (!MS) return TM_EDEVICE;
    hipStream_t cap = MS->cap;
    B.side = MS->side;
    B.fork = MS->fork;
    B.join = MS->join;
    if (capture) {
        TM_HIP(hipStreamSynchronize(st));
        hipGraph_t graph = nullptr;
        tm_status s;
        hipError_t e;
        {
            // no library free (an implicit device synchronisation) during the capture
            std::unique_lock<std::shared_mutex> lk(tm_capture_lock());
            e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return tm_hip_status(e);
            s = mix_enqueue(g, B, cap, true);
            e = hipStreamEndCapture(cap, &graph);
        }
        if (s != TM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        TM_HIP(e);
        e = tm_locked_call([&] { return hipGraphInstantiate(&B.exec, graph, nullptr, nullptr, 0); });
        (void)hipGraphDestroy(graph);
        TM_HIP(e);
        void *tok = tm_prof_begin("count_batch_mixed", st);
        TM_HIP(hipGraphLaunch(B.exec, st));
        tm_prof_end(tok, st);
    } else {
        void *tok = tm_prof_begin("count_batch_mixed", st);
        TM_TRY(mix_enqueue(g, B, st, true));
        tm_prof_end(tok, st);
    }
    std::vector<double> z((size_t)n);
    std::vector<uint64_t> o((size_t)n * 4);
    TM_HIP(hipMemcpyAsync(z.data(), B.z.p, (size_t)n * 8, hipMemcpyDeviceToHost, st));
    TM_HIP(hipMemcpyAsync(o.data(), B.out.p, (size_t)n * 32, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    for (int64_t k = 0; k < n; ++k) {
        est[k] = z[(size_t)k];
        if (kept) {
            kept[k].lo = o[(size_t)(4 * k)];
            kept[k].hi = o[(size_t)(4 * k + 1)];
        }
    }
    return TM_OK;
}

// device bytes tm_batch_mixed allocates for these queries
int64_t tm_batch_mixed_bytes(const tm_graph *g, int64_t n, const int64_t *delta, const int64_t *L) {
    return mix_bytes(g, n, delta, L, 256, nullptr, nullptr, nullptr) + tm_scan_ws_bytes(g->n);
}

void tm_batch_release_thread_ws() {
    MixBufs &b = t_mix;
    for (DevBuf *d : {&b.est, &b.cls_est, &b.kp, &b.wfx, &b.tiles, &b.tnode, &b.qctl, &b.out, &b.z, &b.cnt, &b.tot})
        d->release();
}
