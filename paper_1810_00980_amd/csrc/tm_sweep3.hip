// All 36 three-edge motifs (2 and 3 nodes) in one pass over the per-node
// combined incidence lists.
//
// Every instance (e1, e2, e3) of a 3-edge motif on at most 3 nodes has a
// node x touched by both e1 and e3 (two edges on three nodes share a node).
// In x's time-sorted list L_x (entries: other endpoint y, direction, time),
// e1 is entry i and e3 a later entry j with t_j - t_i <= delta; the middle
// e2 (t_i < t_2 < t_j, strictly) is
//   - another entry of L_x between i and j when e2 also touches x, which is
//     the case for the 2-node motifs and the 3-node stars, or
//   - an edge of the pair {y1, y3} (the triangles),
// so the number of instances with first edge i and last edge j is a count of
// middles of one kind, and all share the duration t_j - t_i (the
// count-duration pairs the sampling framework needs, Sec. 4 and Sec. 5.1).
//
// Forward sweep (anchor = first edge i, scanning j upward) with running
// counters of the middles seen so far, split by direction and by "same other
// endpoint as e1":
//   y_j == y1, x is e1's source:  2-node motifs      (middles with y == y1)
//   y_j == y1:                    stars, e2 elsewhere (middles with y != y1)
//   y_j != y1:                    stars, e2 with e1's (middles with y == y1)
//   y_j != y1:                    triangles           (pair list y1 <-> y_j)
// Backward sweep (anchor = last edge j, scanning i downward) for the stars
// whose middle shares the last edge's other endpoint (middles with y == y3).
// Entries tied in time with the anchor are skipped, and an entry joins the
// middle counters only once the sweep has moved past its time, so tied
// edges never share an instance.  A 2-node instance appears in the lists of
// both of its nodes; it is counted in the list of e1's source only.
//
// Modes: counts only; counts plus the estimator's weighted sum
// sum count * c delta / (c delta - Delta) in 52-bit fixed point (exact
// integer accumulation, so the result does not depend on thread order); or
// counts plus duration histograms (diagnostics).
#include "tm_common.h"

#include <limits.h>

#include "tm_sweep_dev.h"

namespace {

using namespace sweepdev;

// resident waves per SIMD asked of the compiler: the exact triangle sweep is
// latency-bound and would otherwise settle a few registers above five waves
// (at five it takes 95 VGPRs and keeps one 8-byte value per anchor in
// scratch, outside the entry loop); the weighted ones gained nothing from a
// forced count
template <int MODE, bool FWD, unsigned CLS>
constexpr int sweep_waves() {
    return (MODE == MODE_COUNT && FWD && CLS == 8u) ? 5 : 1;
}

template <int MODE, bool FWD, unsigned CLS>
__global__ void __launch_bounds__(SW_TPB) __attribute__((amdgpu_waves_per_eu(sweep_waves<MODE, FWD, CLS>())))
k_sweep3(DevGraph G, SweepArgs a) {
    __shared__ unsigned long long lds[36 * 4];
    for (int k = threadIdx.x; k < 36 * 4; k += SW_TPB) lds[k] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (TM_WAVE - 1);
    // exact triangles run over the ranked sublists
    constexpr bool RANKED = MODE == MODE_COUNT && FWD && CLS == 8u;
    const int64_t *off = RANKED ? G.hi_off : G.inc_off;
    const uint32_t *ndv = RANKED ? G.hi_nd : G.inc_nd;
    const int64_t *tv = RANKED ? G.hi_t : G.inc_t;
    const int64_t nE = RANKED ? G.n_hi : a.n_entries;
    const bool ordered = RANKED && a.order;
    // units: batches of the claim order (heaviest first within each range),
    // or 64-entry chunks in index order
    const int64_t nU = ordered ? a.n_batches : (nE + TM_WAVE - 1) / TM_WAVE;
    const int parts = a.parts;
    int q = (int)(blockIdx.x % (unsigned)parts), left = parts;  // lane 0's range, ranges not yet used up
    while (true) {
        int64_t u = -1;
        if (lane == 0) {
            while (left > 0) {
                const int64_t lo = part_lo(q, nU, parts), hi = part_lo(q + 1, nU, parts);
                const int64_t c = (int64_t)atomicAdd((unsigned long long *)(a.counter + q), 1ull);
                if (lo + c < hi) {
                    u = lo + c;
                    break;
                }
                q = q + 1 == parts ? 0 : q + 1;
                --left;
            }
        }
        u = __shfl(u, 0, TM_WAVE);
        if (u < 0) break;
        const int64_t base = ordered ? (int64_t)a.order[u] * TM_WAVE : u * TM_WAVE;
        int64_t i = base + lane;
        if (i < nE) {
            int64_t x = owner_of(off, G.n, i);
            int64_t lb = off[x], le = off[x + 1];
            uint32_t nd = ndv[i];
            uint32_t y = nd & 0x7FFFFFFFu, d = nd >> 31;
            int64_t t = tv[i];
            bool go = true;
            int64_t wlo = LLONG_MIN, whi = LLONG_MAX;
            unsigned long long *acc = lds;  // where this anchor's sums go
            if (a.windowed == 1) {
                int64_t j = (t - a.s) / a.L + 1;
                go = keep_window(a.seed, (uint64_t)j, a.p);
                wlo = a.s + (j - 1) * a.L;
                whi = a.s + j * a.L - 1;
            } else if (a.windowed == 2) {
                wlo = a.s;
                whi = a.L;
                go = t >= wlo && t <= whi;
            } else if (a.windowed == 3) {
                int64_t j = (t - a.s) / a.L + 1;
                const int32_t kk = a.kidx[j];
                go = kk >= 0;
                wlo = a.s + (j - 1) * a.L;
                whi = a.s + j * a.L - 1;
                if (go) acc = (unsigned long long *)(a.win + (int64_t)kk * 36 * 4);
            }
            if (go) {
                if (FWD) {
                    int64_t hi = (t > LLONG_MAX - a.delta) ? LLONG_MAX : t + a.delta;
                    hi = hi < whi ? hi : whi;
                    if constexpr (RANKED) sweep_tri_ranked(G, a, i, le, y, d, t, hi, wlo, acc);
                    else if constexpr (MODE == MODE_COUNT) {
                        if (G.has_ex) sweep_fwd_prefix(G, a, i, lb, le, (uint32_t)x, y, d, t, hi, acc);
                        else sweep_fwd_count(G, a, i, le, y, d, t, hi, acc);
                    }
                    else sweep_fwd<MODE, CLS>(G, a, i, le, y, d, t, hi, wlo, acc);
                } else {
                    int64_t lo = (t < LLONG_MIN + a.delta) ? LLONG_MIN : t - a.delta;
                    lo = lo > wlo ? lo : wlo;
                    if constexpr (MODE == MODE_COUNT) {
                        if (G.has_ex) sweep_bwd_prefix(G, i, lb, (uint32_t)x, y, d, t, lo, acc);
                        else sweep_bwd_count(G, i, lb, y, d, t, lo, acc);
                    }
                    else sweep_bwd<MODE>(G, a, i, lb, y, d, t, lo, acc);
                }
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 36 * 4; k += SW_TPB) {
        uint64_t v = lds[k];
        if (!v) continue;
        // k = 4*code + {0 count lo, 1 count hi, 2 weight lo, 3 weight hi}
        int part = k & 3;
        uint64_t *o = a.out + (k & ~3);
        if (part == 0) tm_atomic_add_u128(o, o + 1, v, 0);
        else if (part == 1) atomicAdd((unsigned long long *)(o + 1), (unsigned long long)v);
        else if (part == 2) tm_atomic_add_u128(o + 2, o + 3, v, 0);
        else atomicAdd((unsigned long long *)(o + 3), (unsigned long long)v);
    }
}

// p[0 .. n) = 0.  The sweep clears its accumulators and work counters with
// this kernel rather than a memset node, so that a caller may capture the
// whole sequence in a hipGraph and replay it.
__global__ void k_zero_u64(uint64_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

tm_status zero_u64(uint64_t *p, int64_t n, hipStream_t st) {
    if (n <= 0) return TM_OK;
    unsigned nb = tm_blocks(n, 256);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_zero_u64, dim3(nb), dim3(256), 0, st, p, n);
    return tm_hip_status(hipGetLastError());
}

// wfx[d] = round(2^52 L / (L - d)), d = 0..delta: the estimator's weight
// 1 / (1 - d / L) in 52-bit fixed point (at most 2^53 for L >= 2 delta),
// computed exactly by restoring long division of the 116-bit numerator.
__global__ void k_weights_fx(int64_t delta, int64_t L, uint64_t *wfx) {
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d > delta) return;
    uint64_t den = (uint64_t)(L - d);
    uint64_t nhi = (uint64_t)L >> 12, nlo = (uint64_t)L << 52;  // L * 2^52; nhi < den since d <= L/2
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
    if (rem >= den - rem) q += 1;  // round half up
    wfx[d] = q;
}

// Two side streams (default priority) and fork/join events per host thread
// and device.  They are kept until the process ends: destroying them from a
// thread-exit or static destructor could run after the runtime's teardown.
struct SideStreams {
    int dev = -1;
    hipStream_t s[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
};

// nullptr when they cannot be created (the caller then stays on its stream)
SideStreams *side_streams(int dev) {
    thread_local SideStreams per_dev[8];
    if (dev < 0 || dev >= 8) return nullptr;
    SideStreams &S = per_dev[dev];
    if (S.dev != dev) {
        std::shared_lock<std::shared_mutex> lk(tm_capture_lock());
        bool ok = true;
        for (int k = 0; k < 2; ++k) {
            ok = ok && hipStreamCreateWithFlags(&S.s[k], hipStreamNonBlocking) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&S.join[k], hipEventDisableTiming) == hipSuccess;
        }
        ok = ok && hipEventCreateWithFlags(&S.fork, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            return nullptr;
        }
        S.dev = dev;
    }
    return &S;
}

// The four 2-node motifs alone, weighted: grouped by static edge.  Their
// instances lie on one unordered pair, so each anchor (an entry of the
// pair's time-sorted list, i.e. an edge) scans only the later entries of its
// own pair instead of its endpoint's whole list (8x fewer entries on the
// bursty Zipf graphs at delta = 86400).  An entry's direction is the step of
// the a -> b counts at it.  Codes and counters follow the forward sweep:
// e1 = the anchor, x its source; a later entry j (t1 < t_j <= hi) is e3 with
// d3 = 0 when it has e1's direction, and the middles are the entries of
// earlier time groups after t1, split the same way (code 2 d2 + d3).
template <int MODE>
__global__ void __launch_bounds__(SW_TPB) k_pair2(DevGraph G, SweepArgs a) {
    static_assert(MODE == MODE_WEIGHT, "2-node pair sweep is for the weighted pass");
    __shared__ unsigned long long lds[36 * 4];
    for (int k = threadIdx.x; k < 36 * 4; k += SW_TPB) lds[k] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (TM_WAVE - 1);
    const int64_t nE = a.n_entries;  // pair entries, sentinels included
    const PairEnt *E = G.up_ent;
    while (true) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd((unsigned long long *)a.counter, (unsigned long long)TM_WAVE);
        base = __shfl(base, 0, TM_WAVE);
        if (base >= nE) break;
        const int64_t i = base + lane;
        if (i >= nE) continue;
        const PairEnt e1 = E[i];
        if (e1.t == LLONG_MAX) continue;  // a pair's sentinel
        const int64_t t1 = e1.t;
        bool go = true;
        int64_t whi = LLONG_MAX;
        unsigned long long *acc = lds;
        if (a.windowed == 1) {
            const int64_t jw = (t1 - a.s) / a.L + 1;
            go = keep_window(a.seed, (uint64_t)jw, a.p);
            whi = a.s + jw * a.L - 1;
        } else if (a.windowed == 2) {
            go = t1 >= a.s && t1 <= a.L;
            whi = a.L;
        } else if (a.windowed == 3) {
            const int64_t jw = (t1 - a.s) / a.L + 1;
            const int32_t kk = a.kidx[jw];
            go = kk >= 0;
            whi = a.s + jw * a.L - 1;
            if (go) acc = (unsigned long long *)(a.win + (int64_t)kk * 36 * 4);
        }
        if (!go) continue;
        int64_t hi = (t1 > LLONG_MAX - a.delta) ? LLONG_MAX : t1 + a.delta;
        hi = hi < whi ? hi : whi;
        // the entry after the anchor exists (at worst the sentinel)
        int64_t cprev = E[i + 1].c0;
        const int64_t dir1 = cprev - e1.c0;  // 1: a -> b
        Acc<MODE, 4> A;
        A.clear();
        uint64_t cs0 = 0, cs1 = 0, ps0 = 0, ps1 = 0;
        int64_t tg = t1;
        for (int64_t j = i + 1;; j += 4) {
            // four entries and the count after each, loaded together; the
            // sentinel ends every pair, so no load leaves the pair's list + 1
            PairEnt q[4];
            int64_t cn[4];  // the a -> b count after each entry
            bool stop[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = E[j + u < nE ? j + u : nE - 1];
            const int64_t c4 = E[j + 4 < nE ? j + 4 : nE - 1].c0;
#pragma unroll
            for (int u = 0; u < 4; ++u) cn[u] = u < 3 ? q[u + 1].c0 : c4;
            bool done = false;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                stop[u] = done || j + u >= nE || q[u].t == LLONG_MAX || q[u].t > hi;
                done = stop[u];
            }
            uint64_t wq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) wq[u] = stop[u] ? 0 : weight_of<MODE>(a, q[u].t - t1);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (stop[u]) break;
                const int64_t cj = u == 0 ? cprev : cn[u - 1];
                const uint32_t d3 = ((cn[u] - cj) == dir1) ? 0u : 1u;
                const int64_t tj = q[u].t;
                if (tj == t1) continue;
                if (tj != tg) {
                    cs0 += ps0;
                    cs1 += ps1;
                    ps0 = ps1 = 0;
                    tg = tj;
                }
                acc_add<MODE, 4>(A, 0, d3, cs0, wq[u], nullptr, 0, tj - t1, a.delta);
                acc_add<MODE, 4>(A, 2, d3, cs1, wq[u], nullptr, 2, tj - t1, a.delta);
                if (d3) ++ps1;
                else ++ps0;
            }
            if (done) break;
            cprev = cn[3];
        }
        const int codes[4] = {0, 1, 2, 3};
        flush<MODE, 4>(A, codes, acc, nullptr);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 36 * 4; k += SW_TPB) {
        uint64_t v = lds[k];
        if (!v) continue;
        int part = k & 3;
        uint64_t *o = a.out + (k & ~3);
        if (part == 0) tm_atomic_add_u128(o, o + 1, v, 0);
        else if (part == 1) atomicAdd((unsigned long long *)(o + 1), (unsigned long long)v);
        else if (part == 2) tm_atomic_add_u128(o + 2, o + 3, v, 0);
        else atomicAdd((unsigned long long *)(o + 3), (unsigned long long)v);
    }
}

// Claim order of the exact triangle sweep's 64-anchor batches.  Their work
// is heavy-tailed (the longest windows of the ranked sublists: the heaviest
// batch is about three quarters of a wave's fair share of the whole pass),
// so claimed in index order the last heavy batches ran alone at the end.  A
// batch's cost is its first anchor's window length (its lanes' windows are
// nearly equal); keys sort descending.
__global__ void k_tri_batch_cost(DevGraph G, SweepArgs a, int64_t nbt, uint64_t *keys, uint32_t *vals) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbt) return;
    const int64_t i = b * TM_WAVE;
    const int64_t x = owner_of(G.hi_off, G.n, i);
    const int64_t end = G.hi_off[x + 1];
    const int64_t t = G.hi_t[i];
    int64_t hi = (t > LLONG_MAX - a.delta) ? LLONG_MAX : t + a.delta;
    int64_t len = 0;
    if (a.windowed == 2) {
        if (t < a.s || t > a.L) hi = LLONG_MIN;
        else hi = hi < a.L ? hi : a.L;
    }
    if (hi != LLONG_MIN) {
        int64_t lo = i + 1, up = end;  // first entry with time > hi
        while (lo < up) {
            const int64_t mid = (lo + up) >> 1;
            if (G.hi_t[mid] <= hi) lo = mid + 1;
            else up = mid;
        }
        len = lo - (i + 1);
    }
    const uint64_t c = len < 0xFFFFFFFFll ? (uint64_t)len : 0xFFFFFFFFull;
    // the batch's claim range (SweepArgs::parts) above the cost
    int64_t q = (b * a.parts) / nbt;
    while (q > 0 && b < part_lo(q, nbt, a.parts)) --q;
    while (q + 1 < a.parts && b >= part_lo(q + 1, nbt, a.parts)) ++q;
    keys[b] = ((uint64_t)q << 32) | (0xFFFFFFFFull - c);
    vals[b] = (uint32_t)b;
}

// per host thread: keys and batch ids of the claim order
thread_local DevBuf t_order_k, t_order_v;

}  // namespace

void tm_sweep_release_thread_ws() {
    t_order_k.release();
    t_order_v.release();
}

int64_t tm_tri_order_bytes(const tm_graph *g) {
    const int64_t nbt = (g->n_hi + TM_WAVE - 1) / TM_WAVE;
    if (nbt <= 1 || nbt > (int64_t)UINT32_MAX) return 0;
    return nbt * 12 + tm_radix_sort_bytes(nbt);
}

namespace {

tm_status tri_claim_order(const tm_graph *g, SweepArgs &a, hipStream_t st) {
    const DevGraph G = dev_view(g);
    const int64_t nbt = (G.n_hi + TM_WAVE - 1) / TM_WAVE;
    if (nbt <= 1 || nbt > (int64_t)UINT32_MAX) return TM_OK;  // index order
    LoadCacheScope cache;  // the sort's buffers are reused from call to call
    TM_TRY(t_order_k.reserve((size_t)nbt * 8));
    TM_TRY(t_order_v.reserve((size_t)nbt * 4));
    hipLaunchKernelGGL(k_tri_batch_cost, dim3(tm_blocks(nbt, 256)), dim3(256), 0, st, G, a, nbt,
                       t_order_k.as<uint64_t>(), t_order_v.as<uint32_t>());
    TM_HIP(hipGetLastError());
    TM_TRY(tm_radix_sort(t_order_k.as<uint64_t>(), t_order_v.as<uint32_t>(), nbt, 32 + tm_bitlen((uint64_t)a.parts),
                         st));
    a.order = t_order_v.as<uint32_t>();
    a.n_batches = nbt;
    return TM_OK;
}

template <int MODE>
tm_status launch_pair(const tm_graph *g, SweepArgs a, bool fwd, bool bwd, bool single_stream, hipStream_t st) {
    DevGraph G = dev_view(g);
    int dev = g->device, ncu = 0;
    TM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu <= 0) ncu = 256;
    int64_t nE = a.n_entries;
    int64_t want_blocks = (nE + SW_TPB - 1) / SW_TPB;
    int64_t nb = (int64_t)ncu * 8;
    if (nb > want_blocks) nb = want_blocks;
    if (nb < 1) nb = 1;
    static const char *names[3][3] = {{"sweep3_fwd_count", "sweep3_bwd_count", "sweep3_tri_count"},
                                      {"sweep3_fwd_weight", "sweep3_bwd_weight", "sweep3_tri_weight"},
                                      {"sweep3_fwd_hist", "sweep3_bwd_hist", "sweep3_tri_hist"}};
    // The kernels are independent (own work counters, disjoint motif codes)
    // and bound by different things (the 2-node/star sweeps by VALU issue,
    // the triangle sweep by lookup latency), so they run on forked streams
    // and share the CUs; the caller's stream waits for all of them.
    // one claim range per XCD (the grid is dealt to the XCDs in turn) for
    // the exact triangle sweep and its claim order
    a.parts = (ncu % TM_SWEEP_PARTS == 0 && nb >= TM_SWEEP_PARTS) ? TM_SWEEP_PARTS : 1;
    TM_TRY(zero_u64((uint64_t *)a.counter, 3 * TM_SWEEP_PARTS, st));
    if (MODE == MODE_COUNT && fwd && (a.want_fwd & 8u) && a.windowed != 3) TM_TRY(tri_claim_order(g, a, st));
    if (MODE == MODE_WEIGHT && fwd && a.want_fwd == 1u && !bwd) {
        // the 2-node motifs alone: one anchor per pair entry
        SweepArgs b = a;
        b.n_entries = g->m_nl + g->U;
        int64_t nbp = (b.n_entries + SW_TPB - 1) / SW_TPB;
        if (nbp > (int64_t)ncu * 8) nbp = (int64_t)ncu * 8;
        if (nbp < 1) nbp = 1;
        void *tok = tm_prof_begin("pair2_weight", st, tm_prof_pass());
        if constexpr (MODE == MODE_WEIGHT)
            hipLaunchKernelGGL((k_pair2<MODE_WEIGHT>), dim3((unsigned)nbp), dim3(SW_TPB), 0, st, G, b);
        TM_HIP(hipGetLastError());
        tm_prof_end(tok, st);
        return TM_OK;
    }
    struct Launch {
        int kind;  // 0 fwd 2-node/stars, 1 bwd stars, 2 fwd triangles
    } todo[3];
    int nl = 0;
    if (fwd && (a.want_fwd & 8u)) todo[nl++] = {2};
    if (fwd && (a.want_fwd & 7u)) todo[nl++] = {0};
    if (bwd) todo[nl++] = {1};
    if (nl == 0) return TM_OK;
    SideStreams *side = (nl > 1 && !tm_prof_serial() && !single_stream) ? side_streams(dev) : nullptr;
    if (side) {
        TM_HIP(hipEventRecord(side->fork, st));
        for (int k = 1; k < nl; ++k) TM_HIP(hipStreamWaitEvent(side->s[k - 1], side->fork, 0));
    }
    const uint64_t pass = tm_prof_pass();
    // weighted triangles of kept windows over the static triangles first: its
    // set-up (short kernels that read two sizes back) runs before the
    // persistent kernels of the other classes hold the CUs, and its sums then
    // run beside them
    const bool defer_tri = MODE == MODE_WEIGHT && a.static_tri && todo[0].kind == 2;
    if (defer_tri) {
        bool used = false;
        TM_TRY(tm_tri_static_weight(g, a.delta, a.s, a.L, a.seed, a.p, a.windowed == 3 ? a.kidx : nullptr, a.wfx,
                                    a.out, a.windowed == 3 ? a.win : nullptr, st, pass, side != nullptr, &used));
        if (!used) {
            SweepArgs b = a;
            b.counter = a.counter + TM_SWEEP_PARTS * 2;
            b.parts = 1;
            void *tok = tm_prof_begin(names[MODE][2], st, pass);
            hipLaunchKernelGGL((k_sweep3<MODE, true, 8u>), dim3((unsigned)nb), dim3(SW_TPB), 0, st, G, b);
            TM_HIP(hipGetLastError());
            tm_prof_end(tok, st);
        }
    }
    for (int k = 0; k < nl; ++k) {
        hipStream_t sk = (k == 0 || !side) ? st : side->s[k - 1];
        if (k == 0 && defer_tri) continue;
        SweepArgs b = a;
        b.counter = a.counter + TM_SWEEP_PARTS * todo[k].kind;
        // claim ranges by XCD for the exact triangles only (their batches go
        // heaviest first, so a single range scatters every XCD's waves over
        // the whole graph; the weighted sweeps, claimed in index order, ran
        // no faster by XCD ranges in their concurrent pass and slower alone)
        if (!(MODE == MODE_COUNT && todo[k].kind == 2)) b.parts = 1;
        void *tok = tm_prof_begin(names[MODE][todo[k].kind], sk, pass);
        if (todo[k].kind == 0)
            hipLaunchKernelGGL((k_sweep3<MODE, true, 7u>), dim3((unsigned)nb), dim3(SW_TPB), 0, sk, G, b);
        else if (todo[k].kind == 2)
            hipLaunchKernelGGL((k_sweep3<MODE, true, 8u>), dim3((unsigned)nb), dim3(SW_TPB), 0, sk, G, b);
        else
            hipLaunchKernelGGL((k_sweep3<MODE, false, 0u>), dim3((unsigned)nb), dim3(SW_TPB), 0, sk, G, b);
        TM_HIP(hipGetLastError());
        tm_prof_end(tok, sk);
    }
    for (int k = 1; side && k < nl; ++k) {
        TM_HIP(hipEventRecord(side->join[k - 1], side->s[k - 1]));
        TM_HIP(hipStreamWaitEvent(st, side->join[k - 1], 0));
    }
    return TM_OK;
}

// entries scanned by the forward and backward sweeps of every anchor
__global__ void k_census(DevGraph G, int64_t delta, unsigned long long *out) {
    __shared__ unsigned long long sf[SW_TPB], sb[SW_TPB];
    unsigned long long f = 0, b = 0;
    int64_t nE = 2 * G.m_nl;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nE; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t x = owner_of(G.inc_off, G.n, i);
        int64_t lb = G.inc_off[x], le = G.inc_off[x + 1];
        int64_t t = G.inc_t[i];
        int64_t hi = (t > LLONG_MAX - delta) ? LLONG_MAX : t + delta;
        int64_t lo = (t < LLONG_MIN + delta) ? LLONG_MIN : t - delta;
        int64_t a0 = i + 1, a1 = le;  // first entry after i with time > hi
        while (a0 < a1) {
            int64_t mid = (a0 + a1) >> 1;
            if (G.inc_t[mid] <= hi) a0 = mid + 1;
            else a1 = mid;
        }
        int64_t c0 = lb, c1 = i;  // first entry with time >= lo
        while (c0 < c1) {
            int64_t mid = (c0 + c1) >> 1;
            if (G.inc_t[mid] < lo) c0 = mid + 1;
            else c1 = mid;
        }
        f += (unsigned long long)(a0 - i - 1);
        b += (unsigned long long)(i - c0);
    }
    sf[threadIdx.x] = f;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = SW_TPB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sf[threadIdx.x] += sf[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&out[0], sf[0]);
        atomicAdd(&out[1], sb[0]);
    }
}

// binary-search probes of one search over a pair timeline of n entries
__device__ inline unsigned long long search_probes(int64_t n) {
    return n > 0 ? (unsigned long long)(64 - __clzll((unsigned long long)n)) : 0ull;
}

// entries scanned by the exact triangle sweep over the ranked sublists, the
// closing-pair lookups among them, the changes of closing pair and the
// binary-search probes of a plain lookup: per lookup, searches at t_j and
// t_j - delta; per change of pair, one probe to find it and searches at t_i
// and at the window end
__global__ void k_census_ranked(DevGraph G, int64_t delta, unsigned long long *out) {
    __shared__ unsigned long long sh[4][SW_TPB];
    unsigned long long f = 0, lk = 0, pc = 0, pr = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G.n_hi;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t x = owner_of(G.hi_off, G.n, i);
        int64_t le = G.hi_off[x + 1];
        int64_t t = G.hi_t[i];
        uint32_t y1 = G.hi_nd[i] & 0x7FFFFFFFu;
        int64_t hi = (t > LLONG_MAX - delta) ? LLONG_MAX : t + delta;
        uint32_t prev = ~0u;
        unsigned long long lp = 0;  // probes of one search in the current pair
        int64_t j = i + 1;
        for (; j < le && G.hi_t[j] <= hi; ++j) {
            if (G.hi_t[j] == t) continue;
            uint32_t yj = G.hi_nd[j] & 0x7FFFFFFFu;
            if (yj == y1) continue;
            ++lk;
            if (yj != prev) {
                ++pc;
                PairView pv;
                lp = pair_find(G, y1, yj, pv) >= 0 ? search_probes(pv.n) : 0ull;
                pr += 1 + 2 * lp;
            }
            pr += 2 * lp;
            prev = yj;
        }
        f += (unsigned long long)(j - i - 1);
    }
    sh[0][threadIdx.x] = f;
    sh[1][threadIdx.x] = lk;
    sh[2][threadIdx.x] = pc;
    sh[3][threadIdx.x] = pr;
    __syncthreads();
    for (int s = SW_TPB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int q = 0; q < 3; ++q) atomicAdd(&out[2 + q], sh[q][0]);
        atomicAdd(&out[5], sh[3][0]);
    }
}

// the estimate's weighted sweeps for window length L, shift s, seed and p:
// kept anchors, entries scanned forward and backward inside the anchor's
// window, the forward triangle sweep's lookups and pair changes, and the
// binary-search probes of a plain lookup: per lookup, one search at t_j; per
// change of pair, one probe to find it and a search at t_i
__global__ void k_census_est(DevGraph G, int64_t delta, int64_t s, int64_t L, double p, uint64_t seed,
                             unsigned long long *out) {
    __shared__ unsigned long long sh[6][SW_TPB];
    unsigned long long an = 0, f = 0, b = 0, lk = 0, pc = 0, pr = 0;
    int64_t nE = 2 * G.m_nl;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nE; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = G.inc_t[i];
        int64_t jw = (t - s) / L + 1;
        if (!keep_window(seed, (uint64_t)jw, p)) continue;
        ++an;
        int64_t wlo = s + (jw - 1) * L, whi = s + jw * L - 1;
        int64_t x = owner_of(G.inc_off, G.n, i);
        int64_t lb = G.inc_off[x], le = G.inc_off[x + 1];
        uint32_t y1 = G.inc_nd[i] & 0x7FFFFFFFu;
        int64_t hi = (t > LLONG_MAX - delta) ? LLONG_MAX : t + delta;
        hi = hi < whi ? hi : whi;
        int64_t lo = (t < LLONG_MIN + delta) ? LLONG_MIN : t - delta;
        lo = lo > wlo ? lo : wlo;
        uint32_t prev = ~0u;
        unsigned long long lp = 0;
        int64_t j = i + 1;
        for (; j < le && G.inc_t[j] <= hi; ++j) {
            if (G.inc_t[j] == t) continue;
            uint32_t yj = G.inc_nd[j] & 0x7FFFFFFFu;
            if (yj == y1) continue;
            ++lk;
            if (yj != prev) {
                ++pc;
                PairView pv;
                lp = pair_find(G, y1, yj, pv) >= 0 ? search_probes(pv.n) : 0ull;
                pr += 1 + lp;
            }
            pr += lp;
            prev = yj;
        }
        f += (unsigned long long)(j - i - 1);
        int64_t c0 = lb, c1 = i;  // first entry with time >= lo
        while (c0 < c1) {
            int64_t mid = (c0 + c1) >> 1;
            if (G.inc_t[mid] < lo) c0 = mid + 1;
            else c1 = mid;
        }
        b += (unsigned long long)(i - c0);
    }
    sh[0][threadIdx.x] = an;
    sh[1][threadIdx.x] = f;
    sh[2][threadIdx.x] = b;
    sh[3][threadIdx.x] = lk;
    sh[4][threadIdx.x] = pc;
    sh[5][threadIdx.x] = pr;
    __syncthreads();
    for (int w = SW_TPB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < 6; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int q = 0; q < 6; ++q) atomicAdd(&out[q], sh[q][0]);
    }
}

}  // namespace

// L = 0: the exact sweeps (c->anchors and c->tri_anchors set by the
// caller); L > 0: the estimate's weighted sweeps for (s, L, p, seed)
tm_status tm_sweep_census_impl(const tm_graph *g, int64_t delta, int64_t s, int64_t L, double p, uint64_t seed,
                               tm_census *c, hipStream_t st) {
    DevBuf o;
    TM_TRY(o.alloc(64));
    TM_TRY(zero_u64(o.as<uint64_t>(), 6, st));
    unsigned nb = g->m_nl > 0 ? tm_blocks(2 * g->m_nl, SW_TPB) : 1;
    if (nb > 8192) nb = 8192;
    int64_t h[6];
    if (L > 0) {
        if (g->m_nl > 0) {
            hipLaunchKernelGGL(k_census_est, dim3(nb), dim3(SW_TPB), 0, st, dev_view(g), delta, s, L, p, seed,
                               o.as<unsigned long long>());
            TM_HIP(hipGetLastError());
        }
        TM_HIP(hipMemcpyAsync(h, o.p, 48, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        c->anchors = c->tri_anchors = h[0];
        c->fwd_entries = c->tri_entries = h[1];
        c->bwd_entries = h[2];
        c->tri_lookups = h[3];
        c->tri_pairs = h[4];
        c->tri_probes = h[5];
        return TM_OK;
    }
    if (g->m_nl > 0) {
        hipLaunchKernelGGL(k_census, dim3(nb), dim3(SW_TPB), 0, st, dev_view(g), delta, o.as<unsigned long long>());
        TM_HIP(hipGetLastError());
    }
    if (g->n_hi > 0) {
        unsigned nr = tm_blocks(g->n_hi, SW_TPB);
        if (nr > 8192) nr = 8192;
        hipLaunchKernelGGL(k_census_ranked, dim3(nr), dim3(SW_TPB), 0, st, dev_view(g), delta,
                           o.as<unsigned long long>());
        TM_HIP(hipGetLastError());
    }
    TM_HIP(hipMemcpyAsync(h, o.p, 48, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    c->fwd_entries = h[0];
    c->bwd_entries = h[1];
    c->tri_entries = h[2];
    c->tri_lookups = h[3];
    c->tri_pairs = h[4];
    c->tri_probes = h[5];
    return TM_OK;
}

// Motif of each of the 36 codes, in canonical form.
void tm_sweep_code_motif(int code, tm_motif *M) {
    // labels before canonicalisation: x = 0, y1 = 1, third node = 2
    int e[3][2];
    auto ed = [](int (&o)[2], int dir, int a, int b) {  // dir 0: a -> b, 1: b -> a
        o[0] = dir ? b : a;
        o[1] = dir ? a : b;
    };
    int cls = code < 4 ? 0 : code < 12 ? 1 : code < 20 ? 2 : code < 28 ? 3 : 4;
    int r = cls == 0 ? code : (code - 4 - 8 * (cls - 1));
    int d1 = cls == 0 ? 0 : (r >> 2) & 1, d2 = (r >> 1) & 1, d3 = r & 1;
    ed(e[0], d1, 0, 1);
    switch (cls) {
        case 0: ed(e[1], d2, 0, 1); ed(e[2], d3, 0, 1); break;  // 2-node
        case 1: ed(e[1], d2, 0, 2); ed(e[2], d3, 0, 1); break;  // star, middle on a new node
        case 2: ed(e[1], d2, 0, 1); ed(e[2], d3, 0, 2); break;  // star, middle on e1's pair
        case 3: ed(e[1], d2, 1, 2); ed(e[2], d3, 0, 2); break;  // triangle
        default: ed(e[1], d2, 0, 2); ed(e[2], d3, 0, 2); break; // star, middle on e3's pair
    }
    int lab[3] = {-1, -1, -1}, next = 0;
    M->l = 3;
    for (int k = 0; k < 3; ++k) {
        for (int h = 0; h < 2; ++h) {
            int v = e[k][h];
            if (lab[v] < 0) lab[v] = next++;
        }
        M->src[k] = lab[e[k][0]];
        M->dst[k] = lab[e[k][1]];
    }
    M->src[3] = M->dst[3] = 0;
}

int tm_sweep_code_of(const tm_motif *M) {
    if (!M || M->l != 3) return -1;
    for (int c = 0; c < 36; ++c) {
        tm_motif X;
        tm_sweep_code_motif(c, &X);
        bool eq = true;
        for (int k = 0; k < 3; ++k) eq = eq && X.src[k] == M->src[k] && X.dst[k] == M->dst[k];
        if (eq) return c;
    }
    return -1;
}

tm_status tm_fx_weights(int64_t delta, int64_t L, uint64_t *wfx, hipStream_t st) {
    hipLaunchKernelGGL(k_weights_fx, dim3(tm_blocks(delta + 1, 256)), dim3(256), 0, st, delta, L, wfx);
    return tm_hip_status(hipGetLastError());
}

// mode: 0 counts, 1 counts + weights (needs L), 2 counts + histograms.
// out_dev: 36 x 4 u64 (count lo/hi, weight lo/hi), zeroed here.
// hist_dev: 36 x (delta+1) x 2 u64 (mode 2), zeroed here.
tm_status tm_sweep3(const tm_graph *g, uint64_t code_mask_lo, int mode, int64_t delta, int windowed, int64_t s,
                    int64_t L, uint64_t seed, double p, uint64_t *out_dev, uint64_t *hist_dev, uint64_t *wfx_dev,
                    int64_t *counter_dev, hipStream_t st, const int32_t *kidx_dev, uint64_t *win_dev,
                    bool single_stream, bool static_tri) {
    if (windowed == 3 && (!kidx_dev || !win_dev)) return TM_EINVAL;
    SweepArgs a;
    a.kidx = kidx_dev;
    a.win = win_dev;
    a.delta = delta;
    a.windowed = windowed;
    a.s = s;
    a.L = L;
    a.seed = seed;
    a.p = p;
    a.wfx = wfx_dev;
    a.hist = hist_dev;
    a.out = out_dev;
    a.counter = counter_dev;
    a.n_entries = 2 * g->m_nl;
    a.static_tri = static_tri && mode == MODE_WEIGHT && (windowed == 1 || windowed == 3);
    uint32_t wf = 0;
    if (code_mask_lo & 0xFull) wf |= 1;
    if (code_mask_lo & 0xFF0ull) wf |= 2;
    if (code_mask_lo & 0xFF000ull) wf |= 4;
    if (code_mask_lo & 0xFF00000ull) wf |= 8;
    bool bwd = (code_mask_lo >> 28) & 0xFFull;
    a.want_fwd = wf;
    TM_TRY(zero_u64(out_dev, 36 * 4, st));
    if (mode == MODE_HIST) TM_TRY(zero_u64(hist_dev, (int64_t)36 * (delta + 1) * 2, st));
    if (mode == MODE_WEIGHT) {
        hipLaunchKernelGGL(k_weights_fx, dim3(tm_blocks(delta + 1, 256)), dim3(256), 0, st, delta, L, wfx_dev);
        TM_HIP(hipGetLastError());
    }
    if (a.n_entries == 0) return TM_OK;
    switch (mode) {
        case MODE_COUNT: return launch_pair<MODE_COUNT>(g, a, wf != 0, bwd, single_stream, st);
        case MODE_WEIGHT: return launch_pair<MODE_WEIGHT>(g, a, wf != 0, bwd, single_stream, st);
        default: return launch_pair<MODE_HIST>(g, a, wf != 0, bwd, single_stream, st);
    }
}
