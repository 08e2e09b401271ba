// Device side of the three-edge sweep counter, shared by the per-query
// kernels and the batched persistent kernel.  See tm_sweep3.hip for the
// method.
#pragma once

#include "tm_common.h"

#include <limits.h>

namespace sweepdev {

constexpr int SW_TPB = 256;
constexpr int SW_WAVES = SW_TPB / TM_WAVE;

enum : int { MODE_COUNT = 0, MODE_WEIGHT = 1, MODE_HIST = 2 };

struct SweepArgs {
    int64_t delta;
    // windows (estimate): anchor kept when its window's draw is below p
    int32_t windowed;      // 0 none, 1 kept windows of (s, L, seed, p), 2 one window [s, L],
                           // 3 windows with kidx[j] >= 0, summed per window into win
    int64_t s, L;
    uint64_t seed;
    double p;
    const uint64_t *wfx;   // delta+1 fixed-point weights (MODE_WEIGHT)
    uint64_t *hist;        // 36 x (delta+1) x {lo, hi} (MODE_HIST)
    uint64_t *out;         // 36 x {count lo, count hi, weight lo, weight hi}
    int64_t *counter;      // work queue head
    uint32_t want_fwd;     // bit mask: 1 two-node, 2 star B, 4 star A, 8 triangle
    int64_t n_entries;
    const int32_t *kidx;   // windowed 3: kept index of window j (j = 1 .. J), -1 when not kept
    uint64_t *win;         // windowed 3: per kept window, 36 x {count lo, hi, weight lo, hi}
    // exact triangles: the 64-anchor batches of the ranked sublists in the
    // order they are claimed (heaviest window first), or nullptr for index order
    const uint32_t *order = nullptr;
    int64_t n_batches = 0;
    // claims by XCD: the work units (64-entry chunks in index order, or the
    // claim order's batches) form `parts` contiguous ranges (unit u is in
    // range q when ceil(q n / parts) <= u < ceil((q + 1) n / parts)), each
    // with its own counter counter[q]; a work-group starts on the range of
    // its XCD (blockIdx.x mod parts: work-groups are dealt to the XCDs in
    // turn) and moves on to the next range when its own is used up
    int32_t parts = 1;
    // host side: weighted triangles of kept windows over the static triangles
    bool static_tri = false;
};

// first unit of range q of n units in `parts` ranges
__host__ __device__ inline int64_t part_lo(int64_t q, int64_t n, int64_t parts) {
    return (q * n + parts - 1) / parts;
}

__device__ inline void philox10_d(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t a = (uint64_t)0xD2511F53u * x0;
        uint64_t b = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
        uint32_t y2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)b;
        x3 = (uint32_t)a;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ inline bool keep_window(uint64_t seed, uint64_t j, double p) {
    uint32_t x0 = (uint32_t)j, x1 = (uint32_t)(j >> 32), x2 = 0, x3 = 1;
    philox10_d(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
    uint64_t x = ((uint64_t)x1 << 32) | (uint64_t)x0;
    return (double)(x >> 11) * (1.0 / 9007199254740992.0) < p;
}

__device__ inline int64_t owner_of(const int64_t *off, int64_t n, int64_t i) {
    // largest x with off[x] <= i
    int64_t lo = 0, hi = n;  // off[0] = 0 <= i < off[n]
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Unordered pair p = {a < b}: its entries are the edges of both directions,
// time-sorted.  The counts below come as c[0] = a -> b and c[1] = b -> a.

// Lower bound of t in the pair described by m (entries en, n of them): the
// returned index, the a -> b count before it (*c0), and the end of t's
// bucket (*be), past which no entry has time t.  A time in an empty bucket
// is answered from the bucket array alone.
constexpr int PAIR_SCAN = 2;  // entries a search reads together once that few are left

// SCAN: finish with one load of the last PAIR_SCAN entries instead of
// binary steps (shorter dependent chain, more registers)
template <bool SCAN = false>
__device__ inline int64_t pair_lower(const DevGraph &G, const PairMeta &m, const PairEnt *en, int64_t n, int64_t t,
                                     int64_t *c0, int64_t *be) {
    const PairBucket *bk = G.pbk + m.boff;
    if (t <= m.t0) {
        *c0 = 0;
        *be = n;
        return 0;
    }
    int64_t b = (t - m.t0) >> m.shift;
    if (b >= m.nb) {
        *c0 = bk[m.nb].c0;
        *be = n;
        return n;
    }
    // buckets b and b + 1 in one 16-byte load
    PairBucket bb[2];
    __builtin_memcpy(bb, bk + b, sizeof bb);
    *be = bb[1].idx;
    int64_t lo = bb[0].idx, hi = bb[1].idx;
    // c: the a -> b count before entry hi, taken from the bucket or from the
    // last entry the search stepped back to (whole entries are loaded)
    int64_t c = lo == hi ? (int64_t)bb[0].c0 : (int64_t)bb[1].c0;
    while (hi - lo > (SCAN ? PAIR_SCAN : 0)) {
        // branch-free step, so that the entry's time and count arrive in one load
        const int64_t mid = (lo + hi) >> 1;
        const PairEnt q = en[mid];
        const bool before = q.t < t;
        lo = before ? mid + 1 : lo;
        hi = before ? hi : mid;
        c = before ? c : q.c0;
    }
    if (SCAN && lo < hi) {
        // the last few entries are loaded together (index hi is an entry or the
        // pair's sentinel) and the first one not before t is picked
        PairEnt q[PAIR_SCAN];
#pragma unroll
        for (int k = 0; k < PAIR_SCAN; ++k) q[k] = en[lo + k < hi ? lo + k : hi];
        int64_t r = hi;
#pragma unroll
        for (int k = PAIR_SCAN - 1; k >= 0; --k) {
            const bool at = lo + k < hi && !(q[k].t < t);
            r = at ? lo + k : r;
            c = at ? q[k].c0 : c;
        }
        lo = r;
    }
    *c0 = c;
    return lo;
}

// Two lower bounds in one pair with their search steps interleaved, so that
// both searches' loads are in flight together.  r[s] = {index, a -> b count
// before it, bucket end, time of the entry at the index when below the end}.
__device__ inline void pair_lower2(const DevGraph &G, const PairMeta &m, const PairEnt *en, int64_t n, int64_t tA,
                                   int64_t tB, int64_t r[2][4]) {
    const PairBucket *bk = G.pbk + m.boff;
    const int64_t t[2] = {tA, tB};
    int64_t lo[2], hi[2], c[2], th[2], be[2];
    bool early[2], past[2];
    PairBucket bb[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        early[s] = t[s] <= m.t0;
        const int64_t b = early[s] ? 0 : (t[s] - m.t0) >> m.shift;
        past[s] = !early[s] && b >= m.nb;
        __builtin_memcpy(bb[s], bk + (past[s] ? m.nb - 1 : b), sizeof bb[s]);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        if (early[s]) {
            lo[s] = hi[s] = 0;
            c[s] = 0;
            be[s] = n;
            th[s] = m.t0;
        } else if (past[s]) {
            lo[s] = hi[s] = n;
            c[s] = bb[s][1].c0;
            be[s] = n;
            th[s] = 0;
        } else {
            lo[s] = bb[s][0].idx;
            hi[s] = bb[s][1].idx;
            c[s] = lo[s] == hi[s] ? (int64_t)bb[s][0].c0 : (int64_t)bb[s][1].c0;
            be[s] = hi[s];
            th[s] = 0;
        }
    }
    while (lo[0] < hi[0] || lo[1] < hi[1]) {
        PairEnt q[2];
        int64_t mid[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            mid[s] = (lo[s] + hi[s]) >> 1;  // lo when done: an entry or the sentinel
            q[s] = en[mid[s]];
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const bool act = lo[s] < hi[s];
            const bool before = q[s].t < t[s];
            lo[s] = (act && before) ? mid[s] + 1 : lo[s];
            hi[s] = (act && !before) ? mid[s] : hi[s];
            c[s] = (act && !before) ? q[s].c0 : c[s];
            th[s] = (act && !before) ? q[s].t : th[s];
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        r[s][0] = lo[s];
        r[s][1] = c[s];
        r[s][2] = be[s];
        r[s][3] = th[s];
    }
}

// Counts of a pair's entries before t and up to t from t's lower bound r
// (one row of pair_lower2): the entries equal to t, all in t's bucket and
// usually none, are stepped over.
__device__ inline void pair_at_from(const PairEnt *en, const int64_t r[4], int64_t t, int64_t c_lt[2],
                                    int64_t c_le[2]) {
    const int64_t lo = r[0], be = r[2];
    int64_t k = r[1];
    c_lt[0] = k;
    c_lt[1] = lo - k;
    int64_t e = lo;
    if (e < be && r[3] == t) {  // the search read entry lo
        ++e;
        while (e < be && en[e].t == t) ++e;
    }
    if (e != lo) k = en[e].c0;
    c_le[0] = k;
    c_le[1] = e - k;
}

// One pair held in registers for repeated lookups.
struct PairView {
    PairMeta m;
    const PairEnt *en;
    int64_t n;
    __device__ void load(const DevGraph &G, int32_t p) {
        m = G.pmeta[p];
        en = G.up_ent + m.base;
        n = G.pbk[m.boff + m.nb].idx;
    }
    // entries with time < t
    template <bool SCAN = false>
    __device__ void lt(const DevGraph &G, int64_t t, int64_t c[2]) const {
        int64_t k, be;
        int64_t lo = pair_lower<SCAN>(G, m, en, n, t, &k, &be);
        c[0] = k;
        c[1] = lo - k;
    }
    // entries with time <= t (all of them for t = LLONG_MAX)
    template <bool SCAN = false>
    __device__ void le(const DevGraph &G, int64_t t, int64_t c[2]) const {
        int64_t k, be, e;
        if (t == LLONG_MAX) {
            e = n;
            k = G.pbk[m.boff + m.nb].c0;
        } else {
            e = pair_lower<SCAN>(G, m, en, n, t + 1, &k, &be);
        }
        c[0] = k;
        c[1] = e - k;
    }
};

// The pair {u, v}: its id (-1 if no edge joins them), with its metadata
// loaded into pv from the hash slot (one access for both).
__device__ inline int32_t pair_find(const DevGraph &G, uint32_t u, uint32_t v, PairView &pv) {
    uint32_t a = u < v ? u : v, b = u < v ? v : u;
    uint64_t key = ((uint64_t)a << 32) | b;
    int64_t cap = G.ph_cap;
    uint64_t h = tm_pair_hash(key, cap);
    // the slot's 48 bytes of fields as three 16-byte loads issued together;
    // the first probe's fields flow to the result, so none waits for the key
    const uint4 *q = reinterpret_cast<const uint4 *>(G.ph_slot + h);
    uint4 q0 = q[0], q1 = q[1], q2 = q[2];
    // an empty statement that takes the fields as inputs keeps the compiler
    // from sinking their loads behind the key comparison (no code emitted)
    __asm__ volatile("" ::"v"(q1.x), "v"(q1.y), "v"(q1.z), "v"(q1.w), "v"(q2.x), "v"(q2.y), "v"(q2.z), "v"(q2.w),
                     "v"(q0.z), "v"(q0.w));
    uint64_t skey = ((uint64_t)q0.y << 32) | q0.x;
    for (int64_t probe = 1; skey != key && skey != ~0ull && probe < cap; ++probe) {  // collisions (rare)
        h = (h + 1) & (uint64_t)(cap - 1);
        q = reinterpret_cast<const uint4 *>(G.ph_slot + h);
        q0 = q[0];
        q1 = q[1];
        q2 = q[2];
        skey = ((uint64_t)q0.y << 32) | q0.x;
    }
    if (skey != key) return -1;
    pv.m.t0 = (int64_t)(((uint64_t)q0.w << 32) | q0.z);
    pv.m.base = (int64_t)(((uint64_t)q1.y << 32) | q1.x);
    pv.m.boff = (int64_t)(((uint64_t)q1.w << 32) | q1.z);
    pv.m.shift = (int32_t)q2.y;
    pv.m.nb = (int32_t)q2.z;
    pv.en = G.up_ent + pv.m.base;
    pv.n = q2.w;
    return (int32_t)q2.x;
}

// Per-lane accumulator of up to 16 motif codes.
template <int MODE, int NC>
struct Acc {
    uint64_t c[NC];
    uint64_t wl[MODE == MODE_WEIGHT ? NC : 1];
    uint64_t wh[MODE == MODE_WEIGHT ? NC : 1];
    __device__ void clear() {
#pragma unroll
        for (int k = 0; k < NC; ++k) c[k] = 0;
        if constexpr (MODE == MODE_WEIGHT) {
#pragma unroll
            for (int k = 0; k < NC; ++k) wl[k] = wh[k] = 0;
        }
    }
};

// add v at code slot (base + dsel) where dsel in {0,1} is runtime
template <int MODE, int NC>
__device__ inline void acc_add(Acc<MODE, NC> &A, int base, uint32_t dsel, uint64_t v, uint64_t w, uint64_t *hist,
                               int code_base, int64_t dlt, int64_t delta) {
    uint64_t v0 = dsel ? 0 : v, v1 = dsel ? v : 0;
    A.c[base] += v0;
    A.c[base + 1] += v1;
    if constexpr (MODE == MODE_WEIGHT) {
        // (v * w) as 128 bits
        uint64_t plo = v * w;
        uint64_t phi = __umul64hi(v, w);
        uint64_t l0 = dsel ? 0 : plo, h0 = dsel ? 0 : phi;
        uint64_t l1 = dsel ? plo : 0, h1 = dsel ? phi : 0;
        tm_add_u128(A.wl[base], A.wh[base], l0, h0);
        tm_add_u128(A.wl[base + 1], A.wh[base + 1], l1, h1);
    }
    if constexpr (MODE == MODE_HIST) {
        if (hist && v) {
            int64_t code = code_base + dsel;
            uint64_t *h = hist + (code * (delta + 1) + dlt) * 2;
            tm_atomic_add_u128(h, h + 1, v, 0);
        }
    }
}

__device__ inline void lds_add_u128(unsigned long long *lo, unsigned long long *hi, uint64_t vlo, uint64_t vhi) {
    if (vlo) {
        unsigned long long old = atomicAdd(lo, (unsigned long long)vlo);
        if (old + vlo < old) vhi += 1;
    }
    if (vhi) atomicAdd(hi, (unsigned long long)vhi);
}

// Per-lane sums of one motif code (count and weighted sum, 128 bits each),
// used by the batched kernel instead of the shared accumulators.
struct OneCode {
    int32_t code;
    uint64_t cl, ch, wl, wh;
};

template <int MODE, int NC>
__device__ inline void flush(const Acc<MODE, NC> &A, const int *codes, unsigned long long *lds, OneCode *one) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        int code = codes[k];
        if (code < 0) continue;
        if (one) {
            if (code == one->code) {
                tm_add_u128(one->cl, one->ch, A.c[k], 0);
                if constexpr (MODE == MODE_WEIGHT) tm_add_u128(one->wl, one->wh, A.wl[k], A.wh[k]);
            }
            continue;
        }
        if (A.c[k]) lds_add_u128(&lds[4 * code], &lds[4 * code + 1], A.c[k], 0);
        if constexpr (MODE == MODE_WEIGHT) {
            if (A.wl[k] | A.wh[k]) lds_add_u128(&lds[4 * code + 2], &lds[4 * code + 3], A.wl[k], A.wh[k]);
        }
    }
}

template <int MODE>
__device__ inline uint64_t weight_of(const SweepArgs &a, int64_t dlt) {
    if constexpr (MODE == MODE_WEIGHT) return a.wfx[dlt];
    return 0;
}

// add v to tc[4*d1 + 2*d2 + d3] (runtime index, kept in registers)
// Per-lane triangle counts of the eight codes 20 + k in 32 bits: every
// increment is a pair count (below 2^31), so a sum wraps at most once per
// add, and a wrap adds 2^32 to the shared total right away (rare).
struct TriAcc {
    uint32_t c[8];
    unsigned long long *lds;
    OneCode *one;
    __device__ void add(uint32_t idx, uint32_t v);
};

__device__ inline void count_out(unsigned long long *lds, OneCode *one, int code, uint64_t v);

__device__ inline void TriAcc::add(uint32_t idx, uint32_t v) {
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t o = c[k];
        c[k] = o + ((k == idx) ? v : 0u);
        if (c[k] < o) count_out(lds, one, 20 + (int)k, 1ull << 32);
    }
}

// Exact triangle counts at the lowest-ranked node.  Entries i (time ti) and
// j (time tj > ti) of v's list lead to distinct nodes yi, yj that both rank
// above v; every triangle instance with two edges at v has them as (i, j)
// for exactly one of three roles of v, and its third edge lies on the pair
// {yi, yj}:
//   v = x  (shared by first and last edge): middle in (ti, tj)
//   v = y1 (first and middle edge at v):    last edge in (tj, hi]
//   v = y3 (middle and last edge at v):     first edge in [max(tj - delta, lo_win), ti)
// Counting each instance only at its lowest-ranked node counts it once, and
// high-degree nodes, whose lists are long, never do the pair lookups.
// Pair {yi, yc} of the last triangle lookup of an anchor with its counts at
// the anchor's own times, reused while the next entries lead to yc again.
struct TriCache {
    uint32_t yc;
    int32_t p;
    PairView pv;
    int32_t f_ti[2], f_ti1[2], f_hi1[2];  // pair counts (below 2^31)
};

__device__ inline void tri_rank(const DevGraph &G, uint32_t yi, uint32_t di, int64_t ti, uint32_t yj, uint32_t dj,
                                int64_t tj, int64_t hi, int64_t lo_win, int64_t delta, TriAcc &tc, TriCache &C) {
    if (yj != C.yc) {
        C.yc = yj;
        C.p = pair_find(G, yi, yj, C.pv);
        if (C.p >= 0) {
            // counts at ti and up to hi, their lower bounds searched together
            int64_t a0[2], a1[2], h1[2], r[2][4];
            pair_lower2(G, C.pv.m, C.pv.en, C.pv.n, ti, hi == LLONG_MAX ? hi : hi + 1, r);
            pair_at_from(C.pv.en, r[0], ti, a0, a1);
            if (hi == LLONG_MAX) {  // every entry
                r[1][0] = C.pv.n;
                r[1][1] = C.pv.en[C.pv.n].c0;
            }
            h1[0] = r[1][1];
            h1[1] = r[1][0] - r[1][1];
            for (int q = 0; q < 2; ++q) {
                C.f_ti[q] = (int32_t)a0[q];
                C.f_ti1[q] = (int32_t)a1[q];
                C.f_hi1[q] = (int32_t)h1[q];
            }
        }
    }
    if (C.p < 0) return;
    int64_t lo3 = (tj < LLONG_MIN + delta) ? LLONG_MIN : tj - delta;
    lo3 = lo3 > lo_win ? lo3 : lo_win;
    int64_t f_tj[2], f_tj1[2], f_lo3[2];
    {
        // the lower bounds of tj and lo3 searched together
        int64_t r[2][4];
        pair_lower2(G, C.pv.m, C.pv.en, C.pv.n, tj, lo3, r);
        pair_at_from(C.pv.en, r[0], tj, f_tj, f_tj1);
        f_lo3[0] = r[1][1];
        f_lo3[1] = r[1][0] - r[1][1];
    }
    const uint32_t sw = yi > yj ? 1u : 0u;  // index of yi -> yj in the pair's counts
#pragma unroll
    for (uint32_t dir = 0; dir < 2; ++dir) {  // dir 0: yi -> yj, 1: yj -> yi
        const uint32_t k = dir ^ sw;
        // v = x: d1 = di, d2 = dir, d3 = dj
        tc.add(4 * di + 2 * dir + dj, (uint32_t)(f_tj[k] - C.f_ti1[k]));
        // v = y1: d1 = 1 - di, d2 = dj, d3 = dir
        tc.add(4 * (1 - di) + 2 * dj + dir, (uint32_t)(C.f_hi1[k] - f_tj1[k]));
        // v = y3: d1 = 1 - dir, d2 = 1 - di, d3 = 1 - dj
        tc.add(4 * (1 - dir) + 2 * (1 - di) + (1 - dj), (uint32_t)(C.f_ti[k] - f_lo3[k]));
    }
}

// Window scans read U list entries at a time: their times and endpoint
// words load together, then the duration weights of those within the
// horizon are gathered together, so that one memory latency covers U
// entries instead of two per entry; the entries are then visited in order.
// Indices are clamped to the list, so no load leaves it.  (The weighted
// triangle sweep gains too, though it drops from five resident waves to
// four: on a 10M-edge Zipf graph at c 30, p 0.1, 91 -> 84 ms.)
constexpr int SCAN_U = 4;
// The fused forward 2-node/star sweep (all three of its classes in one
// kernel) reads eight at a time: 166 VGPRs instead of 146, still three waves
// per SIMD, and beside the static triangles and the backward sweep the four
// estimate passes on that graph went 109 -> 107 ms.
// The backward sweep at eight takes 106 VGPRs instead of 84 and no longer
// fits beside the other two (120 ms).
constexpr int SCAN_U_FWD = 8;

// forward: entries j = first, first + 1, ... < end (times tv, endpoint words
// ndv) with time <= hi; visit(t, nd, w) with w = the weight of duration
// t - t0 (WEIGHT mode)
template <int MODE, int U, class F>
__device__ inline void scan_up(const int64_t *tv, const uint32_t *ndv, const SweepArgs &a, int64_t first, int64_t end,
                               int64_t t0, int64_t hi, F &&visit) {
    for (int64_t j = first; j < end; j += U) {
        int64_t tq[U];
        uint32_t nq[U];
        uint64_t wq[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = j + u < end ? j + u : end - 1;
            tq[u] = j + u < end ? tv[k] : LLONG_MAX;
            nq[u] = ndv[k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            wq[u] = 0;
            if constexpr (MODE == MODE_WEIGHT) {
                if (tq[u] <= hi) wq[u] = weight_of<MODE>(a, tq[u] - t0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (tq[u] > hi) return;
            visit(tq[u], nq[u], wq[u]);
        }
    }
}

// backward: entries i = last, last - 1, ... >= beg with time >= lo;
// visit(t, nd, w) with w = the weight of duration t0 - t (WEIGHT mode)
template <int MODE, int U, class F>
__device__ inline void scan_down(const DevGraph &G, const SweepArgs &a, int64_t last, int64_t beg, int64_t t0,
                                 int64_t lo, F &&visit) {
    for (int64_t i = last; i >= beg; i -= U) {
        int64_t tq[U];
        uint32_t nq[U];
        uint64_t wq[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = i - u >= beg ? i - u : beg;
            tq[u] = i - u >= beg ? G.inc_t[k] : LLONG_MIN;
            nq[u] = G.inc_nd[k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            wq[u] = 0;
            if constexpr (MODE == MODE_WEIGHT) {
                if (tq[u] >= lo) wq[u] = weight_of<MODE>(a, t0 - tq[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (tq[u] < lo) return;
            visit(tq[u], nq[u], wq[u]);
        }
    }
}

// forward sweep of one anchor (codes 0..27); CLS (1 two-node, 2 star B,
// 4 star A, 8 triangle) fixes at compile time which classes the kernel can
// count, so that a kernel keeps registers only for its own accumulators
template <int MODE, unsigned CLS>
__device__ inline void sweep_fwd(const DevGraph &G, const SweepArgs &a, int64_t i, int64_t end, uint32_t y1,
                                 uint32_t d1, int64_t t1, int64_t hi, int64_t lo_win, unsigned long long *lds,
                                 OneCode *one = nullptr) {
    // slots: 0..3 two-node [2*d2+d3], 4..7 star B, 8..11 star A, 12..15 triangle
    Acc<MODE, 16> A;
    A.clear();
    const bool two = (CLS & 1u) && (a.want_fwd & 1u) && d1 == 0;
    const bool sb = (CLS & 2u) && (a.want_fwd & 2u), sa = (CLS & 4u) && (a.want_fwd & 4u);
    const bool tri = (CLS & 8u) && (a.want_fwd & 8u);
    // Exact triangle totals are counted at the lowest-ranked node instead
    // (sweep_tri_ranked); here triangles are counted only with durations, by
    // one pair lookup per last edge of x's list.
    static_assert(MODE != MODE_COUNT || (CLS & 8u) == 0u, "exact triangles use sweep_tri_ranked");
    TriCache tcache;
    tcache.yc = ~0u;
    tcache.p = -1;
    uint64_t cs0 = 0, cs1 = 0, ca0 = 0, ca1 = 0;  // middles before the current time group
    uint64_t ps0 = 0, ps1 = 0, pa0 = 0, pa1 = 0;  // entries of the current time group
    int64_t tg = t1;
    scan_up<MODE, CLS == 7u ? SCAN_U_FWD : SCAN_U>(G.inc_t, G.inc_nd, a, i + 1, end, t1, hi,
                                                 [&](int64_t tj, uint32_t nd, uint64_t w) {
        if (tj == t1) return;
        if (tj != tg) {
            cs0 += ps0; cs1 += ps1; ca0 += pa0; ca1 += pa1;
            ps0 = ps1 = pa0 = pa1 = 0;
            tg = tj;
        }
        uint32_t yj = nd & 0x7FFFFFFFu, dj = nd >> 31;
        int64_t dlt = tj - t1;
        if (yj == y1) {
            if (two) {
                acc_add<MODE, 16>(A, 0, dj, cs0, w, a.hist, 0, dlt, a.delta);
                acc_add<MODE, 16>(A, 2, dj, cs1, w, a.hist, 2, dlt, a.delta);
            }
            if (sb) {
                acc_add<MODE, 16>(A, 4, dj, ca0 - cs0, w, a.hist, 4 + 4 * (int)d1, dlt, a.delta);
                acc_add<MODE, 16>(A, 6, dj, ca1 - cs1, w, a.hist, 6 + 4 * (int)d1, dlt, a.delta);
            }
            if (dj) ++ps1; else ++ps0;
        } else {
            if (sa) {
                acc_add<MODE, 16>(A, 8, dj, cs0, w, a.hist, 12 + 4 * (int)d1, dlt, a.delta);
                acc_add<MODE, 16>(A, 10, dj, cs1, w, a.hist, 14 + 4 * (int)d1, dlt, a.delta);
            }
            if (tri) {
                // middles on {y1, yj} strictly between t1 and tj; the pair and
                // its count up to t1 are kept while entries lead to yj again
                if (yj != tcache.yc) {
                    tcache.yc = yj;
                    tcache.p = pair_find(G, y1, yj, tcache.pv);
                    if (tcache.p >= 0) {
                        int64_t a1[2];
                        tcache.pv.template le<true>(G, t1, a1);
                        tcache.f_ti1[0] = (int32_t)a1[0];
                        tcache.f_ti1[1] = (int32_t)a1[1];
                    }
                }
                if (tcache.p >= 0) {
                    int64_t up[2];
                    tcache.pv.template lt<true>(G, tj, up);
                    const uint32_t sw = y1 > yj ? 1u : 0u;
                    uint64_t c01 = (uint64_t)(up[sw] - tcache.f_ti1[sw]);
                    uint64_t c10 = (uint64_t)(up[sw ^ 1u] - tcache.f_ti1[sw ^ 1u]);
                    acc_add<MODE, 16>(A, 12, dj, c01, w, a.hist, 20 + 4 * (int)d1, dlt, a.delta);
                    acc_add<MODE, 16>(A, 14, dj, c10, w, a.hist, 22 + 4 * (int)d1, dlt, a.delta);
                }
            }
        }
        if (dj) ++pa1; else ++pa0;
    });
    int codes[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        codes[k] = two ? k : -1;
        codes[4 + k] = 4 + 4 * (int)d1 + k;
        codes[8 + k] = 12 + 4 * (int)d1 + k;
        codes[12 + k] = 20 + 4 * (int)d1 + k;
    }
    flush<MODE, 16>(A, codes, lds, one);
    (void)lo_win;
}

// Exact triangle counts of one anchor i of x's ranked sublist (entries
// [i, end) of hi_nd / hi_t): every later entry j within the horizon that
// leads to another node gives one tri_rank lookup (codes 20..27).
__device__ inline void sweep_tri_ranked(const DevGraph &G, const SweepArgs &a, int64_t i, int64_t end, uint32_t y1,
                                        uint32_t d1, int64_t t1, int64_t hi, int64_t lo_win,
                                        unsigned long long *lds, OneCode *one = nullptr) {
    TriAcc tc;
#pragma unroll
    for (int k = 0; k < 8; ++k) tc.c[k] = 0;
    tc.lds = lds;
    tc.one = one;
    TriCache tcache;
    tcache.yc = ~0u;
    tcache.p = -1;
    for (int64_t j = i + 1; j < end; ++j) {
        int64_t tj = G.hi_t[j];
        if (tj > hi) break;
        if (tj == t1) continue;
        uint32_t nd = G.hi_nd[j];
        uint32_t yj = nd & 0x7FFFFFFFu, dj = nd >> 31;
        if (yj != y1) tri_rank(G, y1, d1, t1, yj, dj, tj, hi, lo_win, a.delta, tc, tcache);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) count_out(lds, one, 20 + k, tc.c[k]);
}

// Exact 2-node and star counts of one forward anchor i (codes 0..19) with
// 32-bit running counts and per-entry work only at the entries that lead to
// y1 ("s-entries").  For window entries j (t1 < tj <= hi, ties with t1
// left out), with cs_k(j) / ca_k(j) the s-entries / all entries of
// direction k in earlier time groups than j:
//   2-node [2k + d]            sum over s-entries j with d_j = d of cs_k(j)      (= Z[d][k])
//   star B [4 + 4 d1 + 2k + d] sum over s-entries j with d_j = d of ca_k - cs_k  (= B[d][k] - Z[d][k])
//   star A [12 + 4 d1 + 2k + d] sum over the other entries j with d_j = d of cs_k(j)
// The star-A sum over all entries, Y[d][k], equals sum over s-entries m of
// direction k of the entries of direction d after m's time group, i.e.
// S_k N_d - U[d][k] with S_k, N_d the window's totals and U[d][k] the sum,
// taken when m's group closes, of the direction-d entries up to that group.
__device__ inline void count_out(unsigned long long *lds, OneCode *one, int code, uint64_t v) {
    if (!v) return;
    if (one) {
        if (one->code == code) tm_add_u128(one->cl, one->ch, v, 0);
    } else {
        lds_add_u128(&lds[4 * code], &lds[4 * code + 1], v, 0);
    }
}

__device__ inline void sweep_fwd_count(const DevGraph &G, const SweepArgs &a, int64_t i, int64_t end, uint32_t y1,
                                       uint32_t d1, int64_t t1, int64_t hi, unsigned long long *lds,
                                       OneCode *one = nullptr) {
    uint32_t as0 = 0, as1 = 0, aa0 = 0, aa1 = 0;  // s-entries / all entries so far, by direction
    uint32_t cs0 = 0, cs1 = 0, ca0 = 0, ca1 = 0;  // the same before the current time group
    uint32_t ps0 = 0, ps1 = 0;                    // s-entries of the current time group
    uint64_t zt0 = 0, zt1 = 0, z10 = 0, z11 = 0;  // sums of cs_k over s-entries: all, and those with d = 1
    uint64_t bt0 = 0, bt1 = 0, b10 = 0, b11 = 0;  // sums of ca_k over s-entries
    uint64_t u00 = 0, u01 = 0, u10 = 0, u11 = 0;  // U[d][k]
    int64_t tg = t1;
    int64_t j = i + 1;
    int64_t tn = j < end ? G.inc_t[j] : 0;
    uint32_t nn = j < end ? G.inc_nd[j] : 0;
    while (j < end) {
        const int64_t tj = tn;
        const uint32_t nd = nn;
        if (tj > hi) break;
        ++j;
        if (j < end) {  // next entry's loads in flight while this one is counted
            tn = G.inc_t[j];
            nn = G.inc_nd[j];
        }
        if (tj == t1) continue;
        if (tj != tg) {
            u00 += (uint64_t)ps0 * aa0;
            u01 += (uint64_t)ps1 * aa0;
            u10 += (uint64_t)ps0 * aa1;
            u11 += (uint64_t)ps1 * aa1;
            ps0 = ps1 = 0;
            cs0 = as0;
            cs1 = as1;
            ca0 = aa0;
            ca1 = aa1;
            tg = tj;
        }
        const uint32_t d = nd >> 31;
        if ((nd & 0x7FFFFFFFu) == y1) {
            zt0 += cs0;
            zt1 += cs1;
            bt0 += ca0;
            bt1 += ca1;
            if (d) {
                z10 += cs0;
                z11 += cs1;
                b10 += ca0;
                b11 += ca1;
                ++as1;
                ++ps1;
            } else {
                ++as0;
                ++ps0;
            }
        }
        aa0 += 1u - d;
        aa1 += d;
    }
    u00 += (uint64_t)ps0 * aa0;
    u01 += (uint64_t)ps1 * aa0;
    u10 += (uint64_t)ps0 * aa1;
    u11 += (uint64_t)ps1 * aa1;
    // Z[d][k], B[d][k], Y[d][k]
    const uint64_t Z00 = zt0 - z10, Z01 = zt1 - z11, Z10 = z10, Z11 = z11;
    const uint64_t B00 = bt0 - b10, B01 = bt1 - b11, B10 = b10, B11 = b11;
    const uint64_t Y00 = (uint64_t)as0 * aa0 - u00, Y01 = (uint64_t)as1 * aa0 - u01;
    const uint64_t Y10 = (uint64_t)as0 * aa1 - u10, Y11 = (uint64_t)as1 * aa1 - u11;
    const int b = 4 * (int)d1;
    if ((a.want_fwd & 1u) && d1 == 0) {  // code 2k + d
        count_out(lds, one, 0, Z00);
        count_out(lds, one, 1, Z10);
        count_out(lds, one, 2, Z01);
        count_out(lds, one, 3, Z11);
    }
    if (a.want_fwd & 2u) {  // code 4 + 4 d1 + 2k + d
        count_out(lds, one, 4 + b, B00 - Z00);
        count_out(lds, one, 5 + b, B10 - Z10);
        count_out(lds, one, 6 + b, B01 - Z01);
        count_out(lds, one, 7 + b, B11 - Z11);
    }
    if (a.want_fwd & 4u) {  // code 12 + 4 d1 + 2k + d
        count_out(lds, one, 12 + b, Y00 - Z00);
        count_out(lds, one, 13 + b, Y10 - Z10);
        count_out(lds, one, 14 + b, Y01 - Z01);
        count_out(lds, one, 15 + b, Y11 - Z11);
    }
}

// Exact star-C counts of one backward anchor (the last edge j, codes 28..35),
// the same way: first edges i (lo <= ti < t3) that lead elsewhere than y3,
// middles the s-entries (leading to y3) strictly between.  Over all i of
// direction d1, the middles after i sum to S_k N_d1 - U[d1][k]; the s-entries'
// own share Z[d1][k] is taken off.
__device__ inline void sweep_bwd_count(const DevGraph &G, int64_t jj, int64_t beg, uint32_t y3, uint32_t d3,
                                       int64_t t3, int64_t lo, unsigned long long *lds, OneCode *one = nullptr) {
    uint32_t as0 = 0, as1 = 0, aa0 = 0, aa1 = 0;
    uint32_t cs0 = 0, cs1 = 0, ps0 = 0, ps1 = 0;
    uint64_t zt0 = 0, zt1 = 0, z10 = 0, z11 = 0;
    uint64_t u00 = 0, u01 = 0, u10 = 0, u11 = 0;
    int64_t tg = t3;
    int64_t i = jj - 1;
    int64_t tn = i >= beg ? G.inc_t[i] : 0;
    uint32_t nn = i >= beg ? G.inc_nd[i] : 0;
    while (i >= beg) {
        const int64_t ti = tn;
        const uint32_t nd = nn;
        if (ti < lo) break;
        --i;
        if (i >= beg) {
            tn = G.inc_t[i];
            nn = G.inc_nd[i];
        }
        if (ti == t3) continue;
        if (ti != tg) {
            u00 += (uint64_t)ps0 * aa0;
            u01 += (uint64_t)ps1 * aa0;
            u10 += (uint64_t)ps0 * aa1;
            u11 += (uint64_t)ps1 * aa1;
            ps0 = ps1 = 0;
            cs0 = as0;
            cs1 = as1;
            tg = ti;
        }
        const uint32_t d = nd >> 31;
        if ((nd & 0x7FFFFFFFu) == y3) {
            zt0 += cs0;
            zt1 += cs1;
            if (d) {
                z10 += cs0;
                z11 += cs1;
                ++as1;
                ++ps1;
            } else {
                ++as0;
                ++ps0;
            }
        }
        aa0 += 1u - d;
        aa1 += d;
    }
    u00 += (uint64_t)ps0 * aa0;
    u01 += (uint64_t)ps1 * aa0;
    u10 += (uint64_t)ps0 * aa1;
    u11 += (uint64_t)ps1 * aa1;
    // code 28 + 4 d1 + 2k + d3 = Y[d1][k] - Z[d1][k]
    const int c = 28 + (int)d3;
    count_out(lds, one, c + 0, (uint64_t)as0 * aa0 - u00 - (zt0 - z10));
    count_out(lds, one, c + 2, (uint64_t)as1 * aa0 - u01 - (zt1 - z11));
    count_out(lds, one, c + 4, (uint64_t)as0 * aa1 - u10 - z10);
    count_out(lds, one, c + 6, (uint64_t)as1 * aa1 - u11 - z11);
}

// Exact 2-node and star counts of a forward anchor from the exact-count
// tables (tm_exact.hip): i is the anchor's position in x's list [lb, le),
// hi its horizon.  With R the entries of the pair P = {x, y1} in (t1, hi],
// R_d those of direction d, and S[d_e*6 + c] the sums over R of the table's
// values c (M_0, M_1, N_0, N_1, N+_0 - M+_0, N+_1 - M+_1):
//   2-node [2k + d]            S[d*6 + k]     - |R_d| M+_k(t1)
//   star B [4 + 4 d1 + 2k + d] S[d*6 + 2 + k] - |R_d| N+_k(t1) - (2-node term)
//   star A [12 + 4 d1 + 2k + d] |R_k| (N+_d(hi) - M+_d(hi)) - S[k*6 + 4 + d]
__device__ inline void ex_counts(const PairView &pv, const DevGraph &G, int64_t t, bool strict, int view,
                                 int64_t *r, int64_t c[2]) {
    int64_t ab[2];
    if (strict) pv.lt(G, t, ab);
    else pv.le(G, t, ab);
    *r = ab[0] + ab[1];
    c[0] = view ? ab[1] : ab[0];  // direction 0 as seen from x
    c[1] = view ? ab[0] : ab[1];
}

__device__ inline void sweep_fwd_prefix(const DevGraph &G, const SweepArgs &a, int64_t i, int64_t lb, int64_t le,
                                        uint32_t x, uint32_t y1, uint32_t d1, int64_t t1, int64_t hi,
                                        unsigned long long *lds, OneCode *one = nullptr) {
    PairView pv;
    (void)pair_find(G, x, y1, pv);  // the anchor's own pair
    const int view = x > y1 ? 1 : 0;
    int64_t r0, r1, Mt1[2], MH[2];
    ex_counts(pv, G, t1, false, view, &r0, Mt1);
    ex_counts(pv, G, hi, false, view, &r1, MH);
    const int64_t *tv = G.inc_t, *c0x = G.ex_c0x;
    int64_t ge = i + 1;
    while (ge < le && tv[ge] == t1) ++ge;
    int64_t u = ge, up = le;  // first entry after hi
    while (u < up) {
        int64_t mid = (u + up) >> 1;
        if (tv[mid] <= hi) u = mid + 1;
        else up = mid;
    }
    const int64_t base0 = c0x[lb];
    const int64_t Nt1[2] = {c0x[ge] - base0, (ge - lb) - (c0x[ge] - base0)};
    const int64_t NH[2] = {c0x[u] - base0, (u - lb) - (c0x[u] - base0)};
    const int64_t R[2] = {MH[0] - Mt1[0], MH[1] - Mt1[1]};
    const uint64_t *row0 = G.ex_rows + ((int64_t)view * G.ex_S + pv.m.base + r0) * 12;
    const uint64_t *row1 = G.ex_rows + ((int64_t)view * G.ex_S + pv.m.base + r1) * 12;
    uint64_t S[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) S[c] = row1[c] - row0[c];
    const int b = 4 * (int)d1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const uint64_t c2 = S[d * 6 + k] - (uint64_t)R[d] * (uint64_t)Mt1[k];
            if ((a.want_fwd & 1u) && d1 == 0) count_out(lds, one, 2 * k + d, c2);
            if (a.want_fwd & 2u)
                count_out(lds, one, 4 + b + 2 * k + d, S[d * 6 + 2 + k] - (uint64_t)R[d] * (uint64_t)Nt1[k] - c2);
            if (a.want_fwd & 4u)
                count_out(lds, one, 12 + b + 2 * k + d,
                          (uint64_t)R[k] * (uint64_t)(NH[d] - MH[d]) - S[k * 6 + 4 + d]);
        }
    }
}

// Star-C counts of a backward anchor (the last edge, time t3) from the
// tables: R' the entries of P = {x, y3} in [lo, t3),
//   code 28 + 4 d1 + 2k + d3 = sum over R'_k of (N_d1 - M_d1)
//                              - |R'_k| (N_d1(lo) - M_d1(lo))
__device__ inline void sweep_bwd_prefix(const DevGraph &G, int64_t j, int64_t lb, uint32_t x, uint32_t y3, uint32_t d3,
                                        int64_t t3, int64_t lo, unsigned long long *lds, OneCode *one = nullptr) {
    PairView pv;
    (void)pair_find(G, x, y3, pv);
    const int view = x > y3 ? 1 : 0;
    int64_t r0, r1, Mlo[2], Mt3[2];
    ex_counts(pv, G, lo, true, view, &r0, Mlo);
    ex_counts(pv, G, t3, true, view, &r1, Mt3);
    const int64_t *tv = G.inc_t, *c0x = G.ex_c0x;
    int64_t u = lb, up = j;  // first entry with time >= lo
    while (u < up) {
        int64_t mid = (u + up) >> 1;
        if (tv[mid] < lo) u = mid + 1;
        else up = mid;
    }
    const int64_t base0 = c0x[lb];
    const int64_t Nlo[2] = {c0x[u] - base0, (u - lb) - (c0x[u] - base0)};
    const uint64_t *row0 = G.ex_rows + ((int64_t)view * G.ex_S + pv.m.base + r0) * 12;
    const uint64_t *row1 = G.ex_rows + ((int64_t)view * G.ex_S + pv.m.base + r1) * 12;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint64_t Rk = (uint64_t)(Mt3[k] - Mlo[k]);
#pragma unroll
        for (int d1 = 0; d1 < 2; ++d1) {
            const uint64_t sn = row1[k * 6 + 2 + d1] - row0[k * 6 + 2 + d1];
            const uint64_t sm = row1[k * 6 + d1] - row0[k * 6 + d1];
            count_out(lds, one, 28 + 4 * d1 + 2 * k + (int)d3, (sn - sm) - Rk * (uint64_t)(Nlo[d1] - Mlo[d1]));
        }
    }
}

// backward sweep of one anchor (codes 28..35): star with e2 on e3's pair
template <int MODE>
__device__ inline void sweep_bwd(const DevGraph &G, const SweepArgs &a, int64_t jj, int64_t beg, uint32_t y3,
                                 uint32_t d3, int64_t t3, int64_t lo, unsigned long long *lds,
                                 OneCode *one = nullptr) {
    // slots [2*d1 + d2]: v is added at slot (2*d1 + d2), d1 runtime -> use base 2*d2 with dsel = d1
    Acc<MODE, 4> A;  // slot index: d2 * 2 + d1
    A.clear();
    uint64_t cs0 = 0, cs1 = 0, ps0 = 0, ps1 = 0;
    int64_t tg = t3;
    scan_down<MODE, SCAN_U>(G, a, jj - 1, beg, t3, lo, [&](int64_t ti, uint32_t nd, uint64_t w) {
        if (ti == t3) return;
        if (ti != tg) {
            cs0 += ps0; cs1 += ps1;
            ps0 = ps1 = 0;
            tg = ti;
        }
        uint32_t yi = nd & 0x7FFFFFFFu, di = nd >> 31;
        if (yi != y3) {
            int64_t dlt = t3 - ti;
            // code 28 + 4*d1 + 2*d2 + d3, kept in slot 2*d2 + d1
            if constexpr (MODE == MODE_HIST) {
                if (cs0) {
                    uint64_t *h = a.hist + ((int64_t)(28 + 4 * di + 0 + d3) * (a.delta + 1) + dlt) * 2;
                    tm_atomic_add_u128(h, h + 1, cs0, 0);
                }
                if (cs1) {
                    uint64_t *h = a.hist + ((int64_t)(28 + 4 * di + 2 + d3) * (a.delta + 1) + dlt) * 2;
                    tm_atomic_add_u128(h, h + 1, cs1, 0);
                }
            }
            acc_add<MODE, 4>(A, 0, di, cs0, w, nullptr, 0, dlt, a.delta);
            acc_add<MODE, 4>(A, 2, di, cs1, w, nullptr, 0, dlt, a.delta);
        } else {
            if (di) ++ps1; else ++ps0;
        }
    });
    int codes[4];
    // slot (2*d2 + d1) -> code 28 + 4*d1 + 2*d2 + d3
    codes[0] = 28 + 0 + 0 + (int)d3;  // d2=0,d1=0
    codes[1] = 28 + 4 + 0 + (int)d3;  // d2=0,d1=1
    codes[2] = 28 + 0 + 2 + (int)d3;  // d2=1,d1=0
    codes[3] = 28 + 4 + 2 + (int)d3;  // d2=1,d1=1
    flush<MODE, 4>(A, codes, lds, one);
}

}  // namespace sweepdev
