// Generic per-window exact counter: backtracking from each anchor edge (the
// motif's first edge) over time-bounded incidence lists.  Motifs of one or
// two edges take one anchor per lane (k_count_generic); longer ones take one
// (anchor, level-1 entry) pair per lane (k_count_split).
//
// For an anchor e1 = (a, b, t1) in a window ending at time W, every later
// motif edge r must have a time in (t_{r-1}, min(t1 + delta, W)] (strictly
// increasing times, inclusive span bound; Sec. 2 instance and duration
// definitions, and the window sub-graph T_j of Algorithm 1).  Level r scans
//   - the (x -> y) pair list when both endpoints of motif edge r are bound,
//   - the out-list of the bound source, or the in-list of the bound
//     destination, keeping entries whose other endpoint is not already the
//     image of a motif node (the node map is a bijection),
// with the start found by binary search on time.  The last level is not
// enumerated for totals: a pair list contributes its range length and a node
// list the number of admissible entries.  With a duration histogram the last
// level is enumerated and each instance adds one to bin t_l - t_1: in a
// block-local u64 histogram in LDS when delta + 1 bins fit (flushed into the
// u128 global bins once per block), else straight into the global bins.  A
// block's LDS bin cannot reach 2^64: that many increments would take
// centuries at the CU's LDS atomic rate.
#include "tm_common.h"

#include <limits.h>

#include "tm_sweep_dev.h"

namespace {

constexpr int CG_TPB = 256;
constexpr int64_t CG_LDS_BINS = TM_GENERIC_LDS_DELTA + 1;  // 64 KB of u64 bins per block

// histogram modes; HM_WEIGHT: no histogram, each instance adds the
// fixed-point weight of its duration (hlo: the delta + 1 weights) to a
// 128-bit per-lane sum, added at the end to hhi[0..1]
constexpr int HM_NONE = 0, HM_GLOBAL = 1, HM_LDS = 2, HM_WEIGHT = 3;

extern __shared__ uint64_t cg_bins[];

struct Acc {
    uint64_t lo, hi;    // instances
    uint64_t wlo, whi;  // HM_WEIGHT: their fixed-point weights
    __device__ void add(uint64_t v) {
        uint64_t s = lo + v;
        hi += (s < lo) ? 1 : 0;
        lo = s;
    }
    __device__ void addw(uint64_t w) {
        uint64_t s = wlo + w;
        whi += (s < wlo) ? 1 : 0;
        wlo = s;
    }
};

// one instance of duration d
template <int HM>
__device__ inline void hist_add(uint64_t *hlo, uint64_t *hhi, int64_t d, Acc &acc) {
    if constexpr (HM == HM_LDS) atomicAdd((unsigned long long *)&cg_bins[d], 1ull);
    else if constexpr (HM == HM_GLOBAL) tm_atomic_add_u128(hlo + d, hhi + d, 1, 0);
    else if constexpr (HM == HM_WEIGHT) acc.addw(hlo[d]);
}

struct Binding {
    int32_t f0, f1, f2, f3, f4;
    __device__ int32_t get(int i) const {
        return i == 0 ? f0 : i == 1 ? f1 : i == 2 ? f2 : i == 3 ? f3 : f4;
    }
    __device__ void set(int i, int32_t w) {
        f0 = (i == 0) ? w : f0;
        f1 = (i == 1) ? w : f1;
        f2 = (i == 2) ? w : f2;
        f3 = (i == 3) ? w : f3;
        f4 = (i == 4) ? w : f4;
    }
    __device__ bool used(int32_t w) const { return w == f0 || w == f1 || w == f2 || w == f3 || w == f4; }
};

// first index in [lo, hi) with t[i] > x
__device__ inline int64_t ub_time(const int64_t *t, int64_t lo, int64_t hi, int64_t x) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (t[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct Range {
    const int32_t *nbr;  // nullptr for pair levels
    const int64_t *t;    // node lists: entry times
    int64_t cur, end;    // node lists: [cur, end) of the list; pairs: of up_ent
    int32_t newnode;     // motif node bound by an entry (-1 for pair levels)
    // pair levels: the unordered pair's entries (both directions, time
    // sorted); an entry runs a -> b (a < b) when the a -> b count steps at it,
    // want = 1 for a -> b, 0 for b -> a; ab = a -> b entries in [cur, end)
    uint32_t want;
    int64_t ab;
};

// Pair level (x -> y) within (tprev, hi]: the unordered pair {x, y} from the
// pair hash, its entries with times in the interval found by two interleaved
// bucket searches, whose a -> b counts also give the directed count.
__device__ inline void open_pair(const DevGraph &G, uint32_t x, uint32_t y, int64_t tprev, int64_t hi, Range &R) {
    R.nbr = nullptr;
    R.t = nullptr;
    R.newnode = -1;
    R.want = x < y ? 1u : 0u;
    R.cur = R.end = 0;
    R.ab = 0;
    sweepdev::PairView pv;
    if (tprev >= hi || G.ph_cap == 0 || sweepdev::pair_find(G, x, y, pv) < 0) return;
    int64_t r[2][4];
    const bool all = hi == LLONG_MAX;  // every entry after tprev
    sweepdev::pair_lower2(G, pv.m, pv.en, pv.n, tprev + 1, all ? tprev + 1 : hi + 1, r);
    const int64_t base = pv.m.base;
    int64_t e = r[1][0], ce = r[1][1];
    if (all) {
        e = pv.n;
        ce = pv.en[pv.n].c0;
    }
    R.cur = base + r[0][0];
    R.end = base + e;
    R.ab = ce - r[0][1];
}

// direction of up_ent entry k: 1 for a -> b
__device__ inline uint32_t pair_dir(const DevGraph &G, int64_t k) {
    return (uint32_t)(G.up_ent[k + 1].c0 - G.up_ent[k].c0);
}

__device__ inline Range open_level(const DevGraph &G, const MotifPlan &P, int r, const Binding &f, int64_t tprev,
                                   int64_t hi) {
    Range R;
    int kind = P.kind[r];
    int64_t lo, up;
    if (kind == LV_PAIR) {
        open_pair(G, (uint32_t)f.get(P.u[r]), (uint32_t)f.get(P.v[r]), tprev, hi, R);
        return R;
    } else if (kind == LV_OUT) {
        int32_t x = f.get(P.u[r]);
        lo = G.out_off[x];
        up = G.out_off[x + 1];
        R.nbr = G.out_nbr;
        R.t = G.out_t;
        R.newnode = P.v[r];
    } else {
        int32_t x = f.get(P.v[r]);
        lo = G.in_off[x];
        up = G.in_off[x + 1];
        R.nbr = G.in_nbr;
        R.t = G.in_t;
        R.newnode = P.u[r];
    }
    R.want = 0;
    R.ab = 0;
    R.cur = ub_time(R.t, lo, up, tprev);
    R.end = ub_time(R.t, R.cur, up, hi);
    return R;
}

template <int HIST>
__device__ inline void count_last(const DevGraph &G, const Range &R, const Binding &f, int64_t t1, Acc &acc,
                                  uint64_t *hlo, uint64_t *hhi) {
    if (R.nbr == nullptr) {
        const int64_t n = R.want ? R.ab : (R.end - R.cur) - R.ab;
        if (HIST && R.cur < R.end) {
            // one 16-byte load per entry: the next entry's count gives this one's direction
            PairEnt e = G.up_ent[R.cur];
            for (int64_t i = R.cur; i < R.end; ++i) {
                const PairEnt nx = G.up_ent[i + 1];
                if ((uint32_t)(nx.c0 - e.c0) == R.want) hist_add<HIST>(hlo, hhi, e.t - t1, acc);
                e = nx;
            }
        }
        acc.add((uint64_t)n);
        return;
    }
    uint64_t c = 0;
    for (int64_t i = R.cur; i < R.end; ++i) {
        if (!f.used(R.nbr[i])) {
            ++c;
            if (HIST) hist_add<HIST>(hlo, hhi, R.t[i] - t1, acc);
        }
    }
    acc.add(c);
}

// Levels R .. LEN-1 below the current binding.
template <int R, int LEN, int HIST>
__device__ inline void levels(const DevGraph &G, const MotifPlan &P, Binding &f, int64_t tprev, int64_t t1,
                              int64_t hi, Acc &acc, uint64_t *hlo, uint64_t *hhi) {
    Range rg = open_level(G, P, R, f, tprev, hi);
    if constexpr (R == LEN - 1) {
        count_last<HIST>(G, rg, f, t1, acc, hlo, hhi);
    } else {
        for (int64_t i = rg.cur; i < rg.end; ++i) {
            if (rg.nbr == nullptr) {
                const PairEnt e = G.up_ent[i];
                if ((uint32_t)(G.up_ent[i + 1].c0 - e.c0) != rg.want) continue;
                levels<R + 1, LEN, HIST>(G, P, f, e.t, t1, hi, acc, hlo, hhi);
            } else {
                int64_t ti = rg.t[i];
                int32_t w = rg.nbr[i];
                if (f.used(w)) continue;
                f.set(rg.newnode, w);
                levels<R + 1, LEN, HIST>(G, P, f, ti, t1, hi, acc, hlo, hhi);
                f.set(rg.newnode, -1);
            }
        }
    }
}

// last time a later motif edge may take: min(t1 + delta, window end)
__device__ inline int64_t anchor_hi(int64_t t1, int64_t delta, int64_t win_end) {
    int64_t hi = (t1 > LLONG_MAX - delta) ? LLONG_MAX : t1 + delta;
    return hi < win_end ? hi : win_end;
}

template <int LEN, int HIST>
__device__ inline void count_anchor(const DevGraph &G, const MotifPlan &P, int64_t pos, int64_t win_end,
                                    int64_t delta, Acc &acc, uint64_t *hlo, uint64_t *hhi) {
    int32_t a = G.es_src[pos], b = G.es_dst[pos];
    if (a == b) return;
    int64_t t1 = G.es_t[pos];
    int64_t hi = anchor_hi(t1, delta, win_end);
    if constexpr (LEN == 1) {
        // every edge of an instance lies in the window, the first one too
        if (t1 <= win_end) {
            acc.add(1);
            if (HIST) hist_add<HIST>(hlo, hhi, 0, acc);
        }
    } else {
        Binding f{-1, -1, -1, -1, -1};
        f.set(0, a);
        f.set(1, b);
        levels<1, LEN, HIST>(G, P, f, t1, t1, hi, acc, hlo, hhi);
    }
}

__device__ inline void wave_reduce_u128(uint64_t &lo, uint64_t &hi) {
#pragma unroll
    for (int o = TM_WAVE / 2; o > 0; o >>= 1) {
        uint64_t olo = __shfl_xor(lo, o, TM_WAVE);
        uint64_t ohi = __shfl_xor(hi, o, TM_WAVE);
        tm_add_u128(lo, hi, olo, ohi);
    }
}

// Persistent waves take 64 consecutive anchors at a time from a global
// counter: per-anchor work is heavy-tailed (hub anchors), so a wave that
// drew light anchors moves on instead of waiting for a static share.
template <int LEN, int HIST>
__global__ void __launch_bounds__(CG_TPB) k_count_generic(DevGraph G, MotifPlan P, int64_t delta, AnchorSet A,
                                                         uint64_t *total, uint64_t *slot_tot, uint64_t *hlo,
                                                         uint64_t *hhi, uint64_t *per_anchor, int32_t *flag,
                                                         unsigned long long *counter) {
    const int64_t nA = A.dev_n ? *A.dev_n : A.n;
    const int lane = threadIdx.x & (TM_WAVE - 1);
    if constexpr (HIST == HM_LDS) {
        for (int64_t k = threadIdx.x; k <= delta; k += blockDim.x) cg_bins[k] = 0;
        __syncthreads();
    }
    uint64_t lo = 0, hi = 0, wlo = 0, whi = 0;
    while (true) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd(counter, (unsigned long long)TM_WAVE);
        base = __shfl(base, 0, TM_WAVE);
        if (base >= nA) break;
        const int64_t i = base + lane;
        if (i >= nA) continue;
        int64_t pos = A.pos ? A.pos[i] : i;
        int64_t we = A.win_end ? A.win_end[i] : LLONG_MAX;
        Acc acc{0, 0, 0, 0};
        count_anchor<LEN, HIST>(G, P, pos, we, delta, acc, hlo, hhi);
        tm_add_u128(lo, hi, acc.lo, acc.hi);
        if constexpr (HIST == HM_WEIGHT) tm_add_u128(wlo, whi, acc.wlo, acc.whi);
        if (per_anchor) {
            per_anchor[i] = acc.lo;
            if (acc.hi) atomicOr(flag, 1);
        }
        if (slot_tot && (acc.lo | acc.hi)) {
            int32_t s = A.slot[i];
            tm_atomic_add_u128(slot_tot + 2 * (int64_t)s, slot_tot + 2 * (int64_t)s + 1, acc.lo, acc.hi);
        }
    }
    wave_reduce_u128(lo, hi);
    if ((threadIdx.x & (TM_WAVE - 1)) == 0 && total) tm_atomic_add_u128(total, total + 1, lo, hi);
    if constexpr (HIST == HM_WEIGHT) {
        wave_reduce_u128(wlo, whi);
        if ((threadIdx.x & (TM_WAVE - 1)) == 0) tm_atomic_add_u128(hhi, hhi + 1, wlo, whi);
    }
    if constexpr (HIST == HM_LDS) {
        __syncthreads();
        for (int64_t k = threadIdx.x; k <= delta; k += blockDim.x) {
            uint64_t v = cg_bins[k];
            if (v) tm_atomic_add_u128(hlo + k, hhi + k, v, 0);
        }
    }
}

// Motifs of three or four edges: the work under one anchor grows with the
// product of its hub degrees, and on hub-heavy graphs a single anchor can
// outweigh a lane's fair share of the whole count many times over.  The
// counter therefore splits each anchor into one work item per entry of its
// level-1 range (the motif's second edge): k_level1_ranges stores each
// anchor's range start and length, an exclusive scan turns the lengths into
// item offsets, and k_count_split's persistent waves claim 64 items at a
// time, find each item's anchor by binary search over the offsets and run
// levels 2 .. LEN-1 under it.  Per-slot and per-anchor outputs are atomic
// adds of the items' counts (their sums equal the per-anchor totals).

struct Level1 {
    const int32_t *nbr;  // nullptr for a pair level (entries of up_ent)
    const int64_t *t;
    int32_t newnode;
};

__device__ inline Level1 level1_list(const DevGraph &G, const MotifPlan &P) {
    if (P.kind[1] == LV_PAIR) return Level1{nullptr, nullptr, -1};
    if (P.kind[1] == LV_OUT) return Level1{G.out_nbr, G.out_t, P.v[1]};
    return Level1{G.in_nbr, G.in_t, P.u[1]};
}

__global__ void __launch_bounds__(CG_TPB) k_level1_ranges(DevGraph G, MotifPlan P, int64_t delta, AnchorSet A,
                                                         int64_t *beg, int64_t *len) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    int64_t pos = A.pos ? A.pos[i] : i;
    int32_t a = G.es_src[pos], b = G.es_dst[pos];
    int64_t s = 0, c = 0;
    if (a != b) {
        int64_t t1 = G.es_t[pos];
        int64_t hi = anchor_hi(t1, delta, A.win_end ? A.win_end[i] : LLONG_MAX);
        Binding f{-1, -1, -1, -1, -1};
        f.set(0, a);
        f.set(1, b);
        Range rg = open_level(G, P, 1, f, t1, hi);
        s = rg.cur;
        c = rg.end - rg.cur;
    }
    beg[i] = s;
    len[i] = c;
}

template <int LEN, int HIST>
__global__ void __launch_bounds__(CG_TPB)
    k_count_split(DevGraph G, MotifPlan P, int64_t delta, AnchorSet A, const int64_t *beg, const int64_t *off,
                  const int64_t *n_items, uint64_t *total, uint64_t *slot_tot, uint64_t *hlo, uint64_t *hhi,
                  uint64_t *per_anchor, int32_t *flag, unsigned long long *counter) {
    static_assert(LEN >= 3, "split counting needs levels below level 1");
    const int64_t T = *n_items, nA = A.n;
    const int lane = threadIdx.x & (TM_WAVE - 1);
    if constexpr (HIST == HM_LDS) {
        for (int64_t k = threadIdx.x; k <= delta; k += blockDim.x) cg_bins[k] = 0;
        __syncthreads();
    }
    const Level1 L1 = level1_list(G, P);
    uint64_t lo = 0, hi = 0, wlo = 0, whi = 0;
    while (true) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd(counter, (unsigned long long)TM_WAVE);
        base = __shfl(base, 0, TM_WAVE);
        if (base >= T) break;
        const int64_t k = base + lane;
        if (k >= T) continue;
        // the item's anchor: the last i with off[i] <= k (anchors with empty
        // ranges share their successor's offset and are never the last)
        int64_t l = 0, h = nA;
        while (h - l > 1) {
            int64_t mid = (l + h) >> 1;
            if (off[mid] <= k) l = mid;
            else h = mid;
        }
        const int64_t i = l;
        const int64_t pos = A.pos ? A.pos[i] : i;
        const int64_t t1 = G.es_t[pos];
        const int64_t thi = anchor_hi(t1, delta, A.win_end ? A.win_end[i] : LLONG_MAX);
        const int64_t j = beg[i] + (k - off[i]);
        Binding f{-1, -1, -1, -1, -1};
        f.set(0, G.es_src[pos]);
        f.set(1, G.es_dst[pos]);
        Acc acc{0, 0, 0, 0};
        bool ok = true;
        int64_t tj;
        if (L1.nbr != nullptr) {
            int32_t w = L1.nbr[j];
            ok = !f.used(w);
            f.set(L1.newnode, w);
            tj = L1.t[j];
        } else {
            // an entry of the pair {x, y} of motif edge 1: only those running x -> y
            const uint32_t x = (uint32_t)f.get(P.u[1]), y = (uint32_t)f.get(P.v[1]);
            ok = pair_dir(G, j) == (x < y ? 1u : 0u);
            tj = G.up_ent[j].t;
        }
        if (ok) levels<2, LEN, HIST>(G, P, f, tj, t1, thi, acc, hlo, hhi);
        if ((acc.lo | acc.hi) == 0) continue;
        tm_add_u128(lo, hi, acc.lo, acc.hi);
        if constexpr (HIST == HM_WEIGHT) tm_add_u128(wlo, whi, acc.wlo, acc.whi);
        if (per_anchor) {
            unsigned long long old = atomicAdd((unsigned long long *)(per_anchor + i), (unsigned long long)acc.lo);
            if (acc.hi || old + acc.lo < old) atomicOr(flag, 1);
        }
        if (slot_tot) {
            int32_t s = A.slot[i];
            tm_atomic_add_u128(slot_tot + 2 * (int64_t)s, slot_tot + 2 * (int64_t)s + 1, acc.lo, acc.hi);
        }
    }
    wave_reduce_u128(lo, hi);
    if (lane == 0 && total) tm_atomic_add_u128(total, total + 1, lo, hi);
    if constexpr (HIST == HM_WEIGHT) {
        wave_reduce_u128(wlo, whi);
        if (lane == 0) tm_atomic_add_u128(hhi, hhi + 1, wlo, whi);
    }
    if constexpr (HIST == HM_LDS) {
        __syncthreads();
        for (int64_t k = threadIdx.x; k <= delta; k += blockDim.x) {
            uint64_t v = cg_bins[k];
            if (v) tm_atomic_add_u128(hlo + k, hhi + k, v, 0);
        }
    }
}

// Per host thread (each call finishes on its stream before returning): the
// work-queue head, and the level-1 range starts, item offsets and item count.
thread_local DevBuf t_cg_counter;
thread_local DevBuf t_cg_items;

template <int LEN, int HIST>
tm_status launch_len(int device, const DevGraph &G, const MotifPlan &P, int64_t delta, const AnchorSet &A,
                     uint64_t *total, uint64_t *slot_tot, uint64_t *hlo, uint64_t *hhi, uint64_t *per_anchor,
                     int32_t *flag, hipStream_t st) {
    int64_t n = A.n;
    if (n <= 0) return TM_OK;
    TM_TRY(t_cg_counter.reserve(8));
    TM_HIP(hipMemsetAsync(t_cg_counter.p, 0, 8, st));
    int ncu = 0;
    TM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
    if (ncu <= 0) ncu = 256;
    int64_t nb = tm_blocks(n, CG_TPB);  // persistent: at most 8 blocks per CU
    if (nb > (int64_t)ncu * 8) nb = (int64_t)ncu * 8;
    size_t lds = HIST == HM_LDS ? (size_t)(delta + 1) * 8 : 0;
    if constexpr (LEN >= 3) {
        TM_TRY(t_cg_items.reserve((size_t)n * 16 + 64));
        int64_t *beg = t_cg_items.as<int64_t>(), *off = beg + n, *n_items = off + n;
        void *tok1 = tm_prof_begin("count_generic_ranges", st);
        hipLaunchKernelGGL(k_level1_ranges, dim3(tm_blocks(n, CG_TPB)), dim3(CG_TPB), 0, st, G, P, delta, A, beg,
                           off);
        tm_status s1 = tm_hip_status(hipGetLastError());
        tm_prof_end(tok1, st);
        TM_TRY(s1);
        TM_TRY(tm_scan_i64(off, n, n_items, st));
        if (per_anchor) TM_HIP(hipMemsetAsync(per_anchor, 0, (size_t)n * 8, st));
        void *tok = tm_prof_begin("count_generic", st);
        hipLaunchKernelGGL((k_count_split<LEN, HIST>), dim3((unsigned)((int64_t)ncu * 8)), dim3(CG_TPB), lds, st, G,
                           P, delta, A, beg, off, n_items, total, slot_tot, hlo, hhi, per_anchor, flag,
                           t_cg_counter.as<unsigned long long>());
        tm_status s = tm_hip_status(hipGetLastError());
        tm_prof_end(tok, st);
        return s;
    } else {
        void *tok = tm_prof_begin("count_generic", st);
        hipLaunchKernelGGL((k_count_generic<LEN, HIST>), dim3((unsigned)nb), dim3(CG_TPB), lds, st, G, P, delta, A,
                           total, slot_tot, hlo, hhi, per_anchor, flag, t_cg_counter.as<unsigned long long>());
        tm_status s = tm_hip_status(hipGetLastError());
        tm_prof_end(tok, st);
        return s;
    }
}

__global__ void k_weight(const uint64_t *hlo, const uint64_t *hhi, int64_t delta, int64_t L, double p, double *out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double sum = 0.0, comp = 0.0;
    for (int64_t d = 0; d <= delta; ++d) {
        uint64_t lo = hlo[d], hi = hhi ? hhi[d] : 0;
        if (lo == 0 && hi == 0) continue;
        double w = (double)L / (double)(L - d);
        double xh = (double)hi;
        double x = xh * 18446744073709551616.0;
        x = x + (double)lo;
        x = x * w;
        double s2 = sum + x;
        if (fabs(sum) >= fabs(x)) comp += (sum - s2) + x;
        else comp += (x - s2) + sum;
        sum = s2;
    }
    out[0] = (sum + comp) / p;
}

}  // namespace

void tm_generic_release_thread_ws() {
    t_cg_counter.release();
    t_cg_items.release();
}

int64_t tm_generic_bytes(int64_t n_anchors, int len) {
    int64_t b = 8;  // the work-queue head
    if (len >= 3 && n_anchors > 0) b += n_anchors * 16 + 64 + tm_scan_ws_bytes(n_anchors);
    return b;
}

tm_status tm_make_plan(const tm_motif *M, MotifPlan *P) {
    if (!M || !P) return TM_EINVAL;
    int l = M->l;
    if (l < 1) return TM_EINVAL;
    if (l > 4) return TM_EUNSUPPORTED;
    // canonical labels: first appearance order, starting with edge 0 = (0, 1)
    int next = 0;
    for (int i = 0; i < l; ++i) {
        int u = M->src[i], v = M->dst[i];
        if (u < 0 || v < 0 || u == v) return TM_EINVAL;
        if (u > next || (u == next && v > next + 1)) return TM_EINVAL;
        if (u == next) ++next;
        if (v > next) return TM_EINVAL;
        if (v == next) ++next;
    }
    P->l = l;
    P->k = next;
    bool bound[5] = {false, false, false, false, false};
    bound[M->src[0]] = bound[M->dst[0]] = true;
    P->kind[0] = LV_PAIR;
    P->u[0] = M->src[0];
    P->v[0] = M->dst[0];
    for (int r = 1; r < 4; ++r) {
        P->kind[r] = LV_PAIR;
        P->u[r] = P->v[r] = 0;
    }
    for (int r = 1; r < l; ++r) {
        int u = M->src[r], v = M->dst[r];
        P->u[r] = u;
        P->v[r] = v;
        if (bound[u] && bound[v]) P->kind[r] = LV_PAIR;
        else if (bound[u]) P->kind[r] = LV_OUT;
        else if (bound[v]) P->kind[r] = LV_IN;
        else return TM_EUNSUPPORTED;  // not prefix-connected
        bound[u] = bound[v] = true;
    }
    return TM_OK;
}

tm_status tm_count_generic(const tm_graph *g, const MotifPlan &P, int64_t delta, const AnchorSet &A, uint64_t *total,
                           uint64_t *slot_tot, uint64_t *hist_lo, uint64_t *hist_hi, uint64_t *per_anchor,
                           int32_t *flag, hipStream_t st) {
    DevGraph G = dev_view(g);
    bool hist = hist_lo != nullptr;
#define TM_LEN_CASE(LN)                                                                                          \
    case LN:                                                                                                     \
        if (!hist)                                                                                               \
            return launch_len<LN, HM_NONE>(g->device, G, P, delta, A, total, slot_tot, nullptr, nullptr,        \
                                           per_anchor, flag, st);                                                \
        if (delta < CG_LDS_BINS)                                                                                 \
            return launch_len<LN, HM_LDS>(g->device, G, P, delta, A, total, slot_tot, hist_lo, hist_hi,         \
                                          per_anchor, flag, st);                                                 \
        return launch_len<LN, HM_GLOBAL>(g->device, G, P, delta, A, total, slot_tot, hist_lo, hist_hi,          \
                                         per_anchor, flag, st);
    switch (P.l) {
        TM_LEN_CASE(1)
        TM_LEN_CASE(2)
        TM_LEN_CASE(3)
        TM_LEN_CASE(4)
        default:
            return TM_EUNSUPPORTED;
    }
#undef TM_LEN_CASE
}

tm_status tm_count_generic_weighted(const tm_graph *g, const MotifPlan &P, int64_t delta, const AnchorSet &A,
                                    uint64_t *total, uint64_t *slot_tot, const uint64_t *wfx, uint64_t *wsum,
                                    hipStream_t st) {
    DevGraph G = dev_view(g);
    uint64_t *w = const_cast<uint64_t *>(wfx);  // read only (the kernels' histogram argument)
    switch (P.l) {
        case 1: return launch_len<1, HM_WEIGHT>(g->device, G, P, delta, A, total, slot_tot, w, wsum, nullptr, nullptr, st);
        case 2: return launch_len<2, HM_WEIGHT>(g->device, G, P, delta, A, total, slot_tot, w, wsum, nullptr, nullptr, st);
        case 3: return launch_len<3, HM_WEIGHT>(g->device, G, P, delta, A, total, slot_tot, w, wsum, nullptr, nullptr, st);
        case 4: return launch_len<4, HM_WEIGHT>(g->device, G, P, delta, A, total, slot_tot, w, wsum, nullptr, nullptr, st);
        default: return TM_EUNSUPPORTED;
    }
}

tm_status tm_weight(const uint64_t *hist_lo, const uint64_t *hist_hi, int64_t delta, int64_t L, double p, double *out,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_weight, dim3(1), dim3(64), 0, st, hist_lo, hist_hi, delta, L, p, out);
    return tm_hip_status(hipGetLastError());
}
