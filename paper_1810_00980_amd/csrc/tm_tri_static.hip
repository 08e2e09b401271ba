// Weighted triangle sums of the estimator over the static triangles.
//
// Every triangle instance (e1, e2, e3) lies on the three unordered pairs of
// one static triangle {u0, u1, u2}, one edge on each pair (Sec. 2: the three
// edges of a 3-node triangle motif join the three node pairs).  Call Q[r] the
// pair opposite u[r].  The first and the last edge share one node s = u[r]
// and the middle edge lies on Q[r]; e1 lies on one of the two other pairs and
// e3 on the remaining one.  Those six roles (r, and which pair holds e1)
// partition the instances.
//
// The estimator (Sec. 4, Algorithm 1) weights each instance inside a kept
// window by a function of its duration t3 - t1 only, so for one role the
// weighted sum over a kept window W is
//   sum over e1 in A, e3 in C with t1 < t3 <= t1 + delta, both in W, of
//   w(t3 - t1) * #{e2 in B : t1 < t2 < t3}
// (A, B, C the role's pair timelines restricted to W).  Only the (e1, e3)
// with at least one middle between them contribute.  A role is driven from
// the lighter of A and C: forward from each e1 (the last edges after the
// first middle past t1), or backward from each e3 (the first edges before the
// last middle ahead of t3), the middles counted by a pointer into B that moves
// with the inner loop.  All reads run along pair timelines that the graph
// stores already sorted, so a (first, last) pair costs one sequential step
// where the per-anchor sweep of the incidence lists needs a hash lookup and a
// bucket search of the pair {y1, y3}.
//
// Work units are (static triangle, kept window) with all three pairs present
// in the window, cut into tasks of at most ST_K driver entries per role.  A
// wave takes one task at a time, in order of decreasing estimated cost, and
// walks its driver entries together; the inner range of each is split over
// the lanes 64 consecutive entries at a time, so that the loads of a step are
// contiguous.  The sums are exact 128-bit integers of the same 52-bit
// fixed-point weights as the incidence-list sweep, so both give the same bits
// (per-lane counts within a task stay below 2^64 because no pair holding 2^28
// entries or more is taken this way).
//
// The static triangles are enumerated once per graph, on first use: pairs are
// oriented from the endpoint with fewer distinct neighbours (ties by id) and
// each node's out-neighbour pairs are checked in the pair hash, which finds
// every triangle once, at its lowest-ranked node.
#include "tm_common.h"

#include <limits.h>
#include <stdlib.h>

#include <mutex>

#include "tm_sweep_dev.h"

namespace {

using namespace sweepdev;

constexpr int ST_TPB = 256;
constexpr int64_t ST_K = 32;  // driver entries per task (on a 10M-edge Zipf graph 16 ran 3% slower, 64 25%)
// candidate out-neighbour pairs the enumeration may check: at most about a
// second's worth, and at most ST_CHECKS_PER_EDGE per edge; and static
// triangles kept: at most one per edge.  Every estimate walks every static
// triangle, while the incidence-list sweep's work follows the kept windows'
// edges, so a graph whose node pairs are nearly all joined (2,000 nodes,
// 4e6 edges: 1.3e9 static triangles, 32 GB) keeps the list sweep, which there
// took 1.7 ms against 275 ms.
constexpr uint64_t ST_MAX_BUILD_CHECKS = 1ull << 33;
constexpr uint64_t ST_CHECKS_PER_EDGE = 64;
// smallest graph (non-self-loop edges) that takes this path by default: the
// set-up costs about fifteen launches and two reads back to the host, about
// a millisecond, which a list sweep of a smaller graph does not
constexpr int64_t ST_MIN_EDGES = (int64_t)1 << 20;
// most windows whose kept ids are listed per call (8 B each); beyond that a
// triangle's walk draws each window it touches instead
constexpr int64_t ST_MAX_WINDOW_LIST = (int64_t)1 << 24;

struct StTri {
    uint32_t u[3];  // nodes, ascending
    int32_t q[3];   // q[r]: pair id of the pair opposite u[r]
};

struct StUnit {
    int64_t lo[3], hi[3];  // entry ranges of Q[0..2] inside the window (absolute, in up_ent)
    int64_t jw;            // window index (1-based, as in the estimator)
    int32_t tri;
    int32_t pad;
};

std::mutex g_st_mu;

__global__ void k_st_zero(uint64_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// endpoints (a < b) of every unordered pair, from its hash slot, and the
// largest pair size
__global__ void k_st_pair_ab(const PairSlot *slots, int64_t cap, uint32_t *pab, unsigned long long *nmax) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    const PairSlot s = slots[i];
    if (s.key == ~0ull || s.id < 0) return;
    pab[2 * (int64_t)s.id] = (uint32_t)(s.key >> 32);
    pab[2 * (int64_t)s.id + 1] = (uint32_t)s.key;
    atomicMax(nmax, (unsigned long long)s.n);
}

// distinct neighbours of every node
__global__ void k_st_deg(const uint32_t *pab, int64_t U, unsigned int *deg) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= U) return;
    atomicAdd(&deg[pab[2 * p]], 1u);
    atomicAdd(&deg[pab[2 * p + 1]], 1u);
}

__device__ inline bool st_ranks_below(const unsigned int *deg, uint32_t a, uint32_t b) {
    return deg[a] < deg[b] || (deg[a] == deg[b] && a < b);
}

// out-degree of every node under the orientation low rank -> high rank
__global__ void k_st_outdeg(const uint32_t *pab, int64_t U, const unsigned int *deg, int64_t *cnt) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= U) return;
    const uint32_t a = pab[2 * p], b = pab[2 * p + 1];
    const uint32_t o = st_ranks_below(deg, a, b) ? a : b;
    atomicAdd((unsigned long long *)&cnt[o], 1ull);
}

__global__ void k_st_outfill(const uint32_t *pab, int64_t U, const unsigned int *deg, int64_t *cur, uint32_t *onbr,
                             int32_t *opid) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= U) return;
    const uint32_t a = pab[2 * p], b = pab[2 * p + 1];
    const bool ab = st_ranks_below(deg, a, b);
    const uint32_t o = ab ? a : b, w = ab ? b : a;
    const int64_t k = (int64_t)atomicAdd((unsigned long long *)&cur[o], 1ull);
    onbr[k] = w;
    opid[k] = (int32_t)p;
}

// candidate checks of the enumeration: sum over nodes of C(out-degree, 2)
__global__ void k_st_checks(const int64_t *off, int64_t n, unsigned long long *tot) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c = 0;
    if (x < n) {
        const uint64_t d = (uint64_t)(off[x + 1] - off[x]);
        c = d * (d > 0 ? d - 1 : 0) / 2;
    }
    for (int o = TM_WAVE / 2; o > 0; o >>= 1) c += __shfl_down(c, o, TM_WAVE);
    if ((threadIdx.x & (TM_WAVE - 1)) == 0 && c) atomicAdd(tot, c);
}

// out-entry e of node u with out-neighbour v: the triangles {u, v, w} for the
// later out-entries w of u joined to v.  FILL writes them at tri[cnt[e]...].
template <bool FILL>
__global__ void k_st_tris(DevGraph G, const int64_t *off, int64_t n, int64_t E, const uint32_t *onbr,
                          const int32_t *opid, int64_t *cnt, StTri *tri) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int64_t u = owner_of(off, n, e);
    const int64_t end = off[u + 1];
    const uint32_t v = onbr[e];
    int64_t c = 0, at = FILL ? cnt[e] : 0;
    for (int64_t j = e + 1; j < end; ++j) {
        const uint32_t w = onbr[j];
        PairView pv;
        const int32_t pvw = pair_find(G, v, w, pv);
        if (pvw < 0) continue;
        ++c;
        if (FILL) {
            // nodes ascending, and the pair opposite each
            uint32_t x[3] = {(uint32_t)u, v, w};
            int32_t opp[3] = {pvw, opid[j], opid[e]};  // opposite u, v, w
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2 - a; ++b)
                    if (x[b] > x[b + 1]) {
                        uint32_t tx = x[b];
                        x[b] = x[b + 1];
                        x[b + 1] = tx;
                        int32_t to = opp[b];
                        opp[b] = opp[b + 1];
                        opp[b + 1] = to;
                    }
            StTri T;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T.u[k] = x[k];
                T.q[k] = opp[k];
            }
            tri[at++] = T;
        }
    }
    if (!FILL) cnt[e] = c;
}

struct StPairs {
    PairMeta m[3];
    const PairEnt *en[3];
    int64_t n[3];
};

__device__ inline void st_pairs(const DevGraph &G, const StTri &T, StPairs &P) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        P.m[r] = G.pmeta[T.q[r]];
        P.en[r] = G.up_ent + P.m[r].base;
        P.n[r] = G.pbk[P.m[r].boff + P.m[r].nb].idx;
    }
}

// first entry of pair r at or after time t (relative index)
__device__ inline int64_t st_lower(const DevGraph &G, const StPairs &P, int r, int64_t t) {
    int64_t c0, be;
    return pair_lower<false>(G, P.m[r], P.en[r], P.n[r], t, &c0, &be);
}

// whether window j is kept: its draw against p, or (kidx) its kept index
__device__ inline bool st_keep(const int32_t *kidx, uint64_t seed, double p, int64_t j) {
    return kidx ? kidx[j] >= 0 : keep_window(seed, (uint64_t)j, p);
}

// kept window ids of the call, ascending: flags, then a scan, then the ids
__global__ void k_st_kept_flags(int64_t J, const int32_t *kidx, uint64_t seed, double p, int64_t *flag) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (j <= J) flag[j - 1] = st_keep(kidx, seed, p, j) ? 1 : 0;
}

__global__ void k_st_kept_fill(int64_t J, const int32_t *kidx, uint64_t seed, double p, const int64_t *pos,
                               int64_t *kept) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (j <= J && st_keep(kidx, seed, p, j)) kept[pos[j - 1]] = j;
}

// The kept windows in which all three pairs of triangle i have entries:
// walked along the lightest pair's entries, from one kept window it touches
// to the next (kept: the call's kept window ids ascending, *nkept of them;
// nullptr: every window it touches, kept by its draw or, with kidx, by its
// kept index).  FILL writes each as a unit at units[uoff[i]...] with its
// task count.
template <bool FILL>
__global__ void k_st_units(DevGraph G, const StTri *tris, int64_t ntri, int64_t s, int64_t L, uint64_t seed,
                           double p, const int32_t *kidx, const int64_t *kept, const int64_t *nkept, int64_t *ucnt,
                           StUnit *units, int64_t *tcnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntri) return;
    const StTri T = tris[i];
    StPairs P;
    st_pairs(G, T, P);
    const int li = (P.n[0] <= P.n[1] && P.n[0] <= P.n[2]) ? 0 : (P.n[1] <= P.n[2] ? 1 : 2);
    int64_t c = 0, at = FILL ? ucnt[i] : 0;
    const int64_t nk = kept ? *nkept : 0;
    int64_t k = 0;
    while (k < P.n[li]) {
        const int64_t t = P.en[li][k].t;
        const int64_t jw = (t - s) / L + 1;
        if (kept) {
            // the first kept window at or after jw; entries before it are skipped
            int64_t a = 0, b = nk;
            while (a < b) {
                const int64_t mid = (a + b) >> 1;
                if (kept[mid] < jw) a = mid + 1;
                else b = mid;
            }
            if (a == nk) break;
            if (kept[a] != jw) {
                k = st_lower(G, P, li, s + (kept[a] - 1) * L);
                continue;
            }
        }
        const int64_t wlo = s + (jw - 1) * L, whi = wlo > LLONG_MAX - L ? LLONG_MAX - 1 : wlo + L - 1;
        const int64_t kn = st_lower(G, P, li, whi + 1);
        if (kept || st_keep(kidx, seed, p, jw)) {
            int64_t lo[3], hi[3];
            bool all = true;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                if (r == li) {
                    lo[r] = k;
                    hi[r] = kn;
                } else {
                    lo[r] = st_lower(G, P, r, wlo);
                    hi[r] = st_lower(G, P, r, whi + 1);
                }
                all = all && hi[r] > lo[r];
            }
            if (all) {
                if (FILL) {
                    StUnit u;
                    int64_t nt = 0;
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        u.lo[r] = P.m[r].base + lo[r];
                        u.hi[r] = P.m[r].base + hi[r];
                    }
                    u.jw = jw;
                    u.tri = (int32_t)i;
                    u.pad = 0;
#pragma unroll
                    for (int role = 0; role < 6; ++role) {
                        const int r = role >> 1, o = role & 1;
                        const int r1 = o ? (r + 2) % 3 : (r + 1) % 3, r3 = o ? (r + 1) % 3 : (r + 2) % 3;
                        const int64_t nA = hi[r1] - lo[r1], nC = hi[r3] - lo[r3];
                        const int64_t nd = nA <= nC ? nA : nC;
                        nt += (nd + ST_K - 1) / ST_K;
                    }
                    units[at] = u;
                    tcnt[at] = nt;
                    ++at;
                }
                ++c;
            }
        }
        k = kn;
    }
    if (!FILL) ucnt[i] = c;
}

// One task word per (unit, role, chunk of driver entries) and its sort key:
// the estimated work (driver entries times the other pair's entries within
// delta of each), inverted so that an ascending sort puts the heaviest first.
__global__ void k_st_tasks(const StUnit *units, int64_t nu, const int64_t *toff, int64_t delta, int64_t L,
                           uint64_t *tasks, uint64_t *keys, uint32_t *vals) {
    int64_t ui = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ui >= nu) return;
    const StUnit u = units[ui];
    int64_t at = toff[ui];
    const double dens = (double)delta / (double)L;
    for (int role = 0; role < 6; ++role) {
        const int r = role >> 1, o = role & 1;
        const int r1 = o ? (r + 2) % 3 : (r + 1) % 3, r3 = o ? (r + 1) % 3 : (r + 2) % 3;
        const int64_t nA = u.hi[r1] - u.lo[r1], nC = u.hi[r3] - u.lo[r3];
        const int64_t nd = nA <= nC ? nA : nC, no = nA <= nC ? nC : nA;
        for (int64_t ch = 0; ch * ST_K < nd; ++ch) {
            const int64_t k = nd - ch * ST_K < ST_K ? nd - ch * ST_K : ST_K;
            double cost = (double)k * (1.0 + (double)no * dens);
            if (cost > 4294967295.0) cost = 4294967295.0;
            tasks[at] = (uint64_t)ui | ((uint64_t)role << 32) | ((uint64_t)ch << 35);
            keys[at] = 0xFFFFFFFFull - (uint64_t)cost;
            vals[at] = (uint32_t)at;
            ++at;
        }
    }
}

// first index k' in [k, e) whose time is after x (GE: not before x), given
// that every index below k is before it; e when none.  Steps of growing
// length, then a binary search: a pointer that moves little costs little.
template <bool GE>
__device__ inline int64_t st_seek(const PairEnt *E, int64_t k, int64_t e, int64_t x) {
    auto before = [&](int64_t idx) {
        const int64_t t = E[idx].t;
        return GE ? t < x : t <= x;
    };
    if (k >= e || !before(k)) return k;
    int64_t lo = k, hi = e, step = 1;
    while (true) {
        const int64_t nx = lo + step;
        if (nx >= e) break;
        if (!before(nx)) {
            hi = nx;
            break;
        }
        lo = nx;
        step <<= 1;
    }
    while (hi - lo > 1) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (before(mid)) lo = mid;
        else hi = mid;
    }
    return hi;
}

// direction of pair entry i relative to node s of the pair {s, o}: 0 when s
// is the source (entry c0 counts the edges min -> max before it)
__device__ inline uint32_t st_dir(const PairEnt &cur, const PairEnt &next, bool s_is_min) {
    const uint32_t ab = (uint32_t)(next.c0 - cur.c0);  // 1: min -> max
    return s_is_min ? 1u - ab : ab;
}

struct StArgs {
    int64_t delta, s, L;
    const uint64_t *wfx;
    const StTri *tris;
    const StUnit *units;
    const uint64_t *tasks;
    const uint32_t *order;
    int64_t ntask;
    unsigned long long *counter;
    uint64_t *out;  // 36 x {count lo, hi, weight lo, hi}; codes 20..27 are added to
    // per-window sums instead: window j's kept index kidx[j] picks its 36 x 4
    // slot of win (nullptr: the shared sums of out)
    const int32_t *kidx;
    uint64_t *win;
};

// first index k' in [lo, k] such that every index in [k', k) has a time after
// x, i.e. the first index after x when walking down from k (k itself is after
// x or the end); indexes below lo are not read.
__device__ inline int64_t st_seek_down(const PairEnt *E, int64_t lo, int64_t k, int64_t x) {
    if (k <= lo || E[k - 1].t <= x) return k;
    int64_t hi = k - 1, bad = lo - 1, step = 1;  // E[hi].t > x; bad: known not after x (or lo - 1)
    while (true) {
        const int64_t nx = hi - step;
        if (nx < lo) break;
        if (E[nx].t <= x) {
            bad = nx;
            break;
        }
        hi = nx;
        step <<= 1;
    }
    while (hi - bad > 1) {
        const int64_t mid = bad + ((hi - bad) >> 1);
        if (E[mid].t > x) hi = mid;
        else bad = mid;
    }
    return hi;
}

using StAcc = Acc<MODE_WEIGHT, 4>;

// One first edge (time t1) driving forward: its last edges C[j0 ..] with
// times up to hi, 64 per step, one per lane (consecutive entries: the loads
// of a step are contiguous).  Middles before t3 come from the first middle
// index not before the step's first time, shared by the wave, unless a
// middle falls inside the step's span (then the lane seeks its own).  Slots:
// 2 dm + d3 (dm: middle direction, 0 for y1 -> z).
// CENSUS: count the steps and the valid lanes instead (cnt[1], cnt[2]).
template <bool CENSUS>
__device__ inline void st_fwd_entry(const PairEnt *E, int lane, int64_t t1, int64_t hi, int64_t j0, int64_t hiC,
                                    int64_t b1, int64_t hiB, int64_t cb1, bool s_min_c, bool y1_min,
                                    const uint64_t *wfx, StAcc &A, uint64_t *cnt) {
    int64_t pbase = b1;
    for (int64_t js = j0;; js += TM_WAVE) {
        const int64_t j = js + lane;
        PairEnt ec;
        ec.t = LLONG_MAX;
        ec.c0 = 0;
        if (j <= hiC) ec = E[j];  // index hiC is the next pair entry or the sentinel
        const bool valid = j < hiC && ec.t <= hi;
        const unsigned long long vm = __ballot(valid);
        if (vm == 0ull) break;  // valid lanes form a prefix
        if constexpr (CENSUS) {
            cnt[1] += 1;
            cnt[2] += (uint64_t)__popcll(vm);
            if (!(vm >> (TM_WAVE - 1))) break;
            continue;
        }
        int64_t nc0 = __shfl_down(ec.c0, 1, TM_WAVE);
        if (lane == TM_WAVE - 1 && valid) nc0 = E[j + 1].c0;
        const int64_t t3 = ec.t;
        pbase = st_seek<true>(E, pbase, hiB, __shfl(t3, 0, TM_WAVE));
        const PairEnt ebp = E[pbase];
        if (valid) {
            int64_t pb = pbase, cpb = ebp.c0;
            if (ebp.t < t3) {  // a middle inside the step's span
                pb = st_seek<true>(E, pbase + 1, hiB, t3);
                cpb = E[pb].c0;
            }
            const uint64_t ntot = (uint64_t)(pb - b1), nab = (uint64_t)(cpb - cb1);
            const uint64_t m0 = y1_min ? nab : ntot - nab;
            const uint32_t ab = (uint32_t)(nc0 - ec.c0);
            const uint32_t d3 = s_min_c ? 1u - ab : ab;
            const uint64_t w = wfx[t3 - t1];
            acc_add<MODE_WEIGHT, 4>(A, 0, d3, m0, w, nullptr, 0, 0, 0);
            acc_add<MODE_WEIGHT, 4>(A, 2, d3, ntot - m0, w, nullptr, 0, 0, 0);
        }
        if (!(vm >> (TM_WAVE - 1))) break;
    }
}

// One last edge (time t3) driving backward: its first edges A[i0 - 1], A[i0 -
// 2], ... with times from lo on, 64 per step.  The first middle after t1 is
// shared by the wave from the step's latest first edge unless a middle falls
// inside the step's span.  Slots: 2 dm + d1.
template <bool CENSUS>
__device__ inline void st_bwd_entry(const PairEnt *E, int lane, int64_t t3, int64_t lo, int64_t i0, int64_t loA,
                                    int64_t pb, int64_t loB, int64_t cbt, bool s_min_a, bool y1_min,
                                    const uint64_t *wfx, StAcc &A, uint64_t *cnt) {
    int64_t qbase = pb;
    for (int64_t is = i0 - 1;; is -= TM_WAVE) {
        const int64_t i = is - lane;
        PairEnt ea;
        ea.t = LLONG_MIN;
        ea.c0 = 0;
        if (i >= loA) ea = E[i];
        const bool valid = i >= loA && ea.t >= lo;
        const unsigned long long vm = __ballot(valid);
        if (vm == 0ull) break;
        if constexpr (CENSUS) {
            cnt[1] += 1;
            cnt[2] += (uint64_t)__popcll(vm);
            if (!(vm >> (TM_WAVE - 1))) break;
            continue;
        }
        int64_t nc0 = __shfl_up(ea.c0, 1, TM_WAVE);  // lane - 1 holds entry i + 1
        if (lane == 0) nc0 = E[i + 1].c0;             // i + 1 <= i0 <= hiA
        const int64_t t1 = ea.t;
        qbase = st_seek_down(E, loB, qbase, __shfl(t1, 0, TM_WAVE));
        const int64_t tq = qbase > loB ? E[qbase - 1].t : LLONG_MIN;
        const int64_t cq = E[qbase].c0;
        if (valid) {
            int64_t qb = qbase, cqb = cq;
            if (tq > t1) {  // a middle inside the step's span
                qb = st_seek_down(E, loB, qbase, t1);
                cqb = E[qb].c0;
            }
            const uint64_t ntot = (uint64_t)(pb - qb), nab = (uint64_t)(cbt - cqb);
            const uint64_t m0 = y1_min ? nab : ntot - nab;
            const uint32_t ab = (uint32_t)(nc0 - ea.c0);
            const uint32_t d1 = s_min_a ? 1u - ab : ab;
            const uint64_t w = wfx[t3 - t1];
            acc_add<MODE_WEIGHT, 4>(A, 0, d1, m0, w, nullptr, 0, 0, 0);
            acc_add<MODE_WEIGHT, 4>(A, 2, d1, ntot - m0, w, nullptr, 0, 0, 0);
        }
        if (!(vm >> (TM_WAVE - 1))) break;
    }
}

__device__ inline void st_flush(const StAcc &A, const int codes[4], unsigned long long *lds) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = codes[k];
        if (A.c[k]) lds_add_u128(&lds[4 * c], &lds[4 * c + 1], A.c[k], 0);
        if (A.wl[k] | A.wh[k]) lds_add_u128(&lds[4 * c + 2], &lds[4 * c + 3], A.wl[k], A.wh[k]);
    }
}

// The four sums of every lane added over the wave, then by lane 0 into a
// window's slot in device memory (per-lane counts of a task stay below 2^55,
// so the wave's count sum needs no carry).
__device__ inline void st_flush_global(const StAcc &A, const int codes[4], uint64_t *dst, int lane) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint64_t c = A.c[k], wl = A.wl[k], wh = A.wh[k];
        for (int off = TM_WAVE / 2; off > 0; off >>= 1) {
            const uint64_t oc = __shfl_xor(c, off, TM_WAVE);
            const uint64_t ol = __shfl_xor(wl, off, TM_WAVE);
            const uint64_t oh = __shfl_xor(wh, off, TM_WAVE);
            c += oc;
            const uint64_t nl = wl + ol;
            wh += oh + (nl < wl ? 1ull : 0ull);
            wl = nl;
        }
        if (lane == 0) {
            uint64_t *o = dst + 4 * codes[k];
            if (c) tm_atomic_add_u128(o, o + 1, c, 0);
            if (wl | wh) tm_atomic_add_u128(o + 2, o + 3, wl, wh);
        }
    }
}

// One task, by the whole wave: the driver entries one after another (every
// lane computes the same pointers), the inner ranges 64 entries at a time.
// Sums go to two accumulator sets chosen by the driver entry's direction
// (the same for every lane), flushed once per task.
template <bool CENSUS>
__device__ void st_task(const DevGraph &G, const StArgs &a, uint64_t tw, int lane, unsigned long long *lds,
                        uint64_t *cnt) {
    const StUnit u = a.units[(uint32_t)tw];
    const int role = (int)((tw >> 32) & 7u);
    const int64_t chunk = (int64_t)(tw >> 35);
    const StTri T = a.tris[u.tri];
    const int r = role >> 1, o = role & 1;
    const int r1 = o ? (r + 2) % 3 : (r + 1) % 3, r3 = o ? (r + 1) % 3 : (r + 2) % 3;
    // shared node s, e1 on {s, y1} = Q[r1], e3 on {s, z} = Q[r3], e2 on {y1, z} = Q[r]
    const uint32_t sN = T.u[r], y1 = T.u[r3], z = T.u[r1];
    const int64_t loA = u.lo[r1], hiA = u.hi[r1], loB = u.lo[r], hiB = u.hi[r], loC = u.lo[r3], hiC = u.hi[r3];
    const int64_t wlo = a.s + (u.jw - 1) * a.L, whi = wlo > LLONG_MAX - a.L ? LLONG_MAX - 1 : wlo + a.L - 1;
    const PairEnt *E = G.up_ent;
    const bool s_min_a = sN < y1, s_min_c = sN < z, y1_min = y1 < z;
    StAcc A0, A1;
    A0.clear();
    A1.clear();
    const bool fwd = hiA - loA <= hiC - loC;
    if (fwd) {
        const int64_t d0 = loA + chunk * ST_K, d1e = d0 + ST_K < hiA ? d0 + ST_K : hiA;
        int64_t b1 = loB, j0 = loC;
        for (int64_t i = d0; i < d1e; ++i) {
            const PairEnt ea = E[i];
            const int64_t t1 = ea.t;
            int64_t hi = (t1 > LLONG_MAX - a.delta) ? LLONG_MAX : t1 + a.delta;
            hi = hi < whi ? hi : whi;
            b1 = st_seek<false>(E, b1, hiB, t1);  // first middle after t1
            if (b1 == hiB) break;
            const PairEnt eb1 = E[b1];
            if (eb1.t >= hi) continue;
            j0 = st_seek<false>(E, j0, hiC, eb1.t);  // first last edge after it
            if (j0 == hiC) break;
            const uint32_t d1 = st_dir(ea, E[i + 1], s_min_a);
            cnt[0] += 1;
            if (d1) st_fwd_entry<CENSUS>(E, lane, t1, hi, j0, hiC, b1, hiB, eb1.c0, s_min_c, y1_min, a.wfx, A1, cnt);
            else st_fwd_entry<CENSUS>(E, lane, t1, hi, j0, hiC, b1, hiB, eb1.c0, s_min_c, y1_min, a.wfx, A0, cnt);
        }
        if constexpr (CENSUS) return;
        // set d1, slot 2 dm + d3 -> code 20 + 4 d1 + 2 dm + d3
        const int c0[4] = {20, 21, 22, 23}, c1[4] = {24, 25, 26, 27};
        if (a.kidx) {
            uint64_t *dst = a.win + (int64_t)a.kidx[u.jw] * 36 * 4;
            st_flush_global(A0, c0, dst, lane);
            st_flush_global(A1, c1, dst, lane);
        } else {
            st_flush(A0, c0, lds);
            st_flush(A1, c1, lds);
        }
    } else {
        const int64_t d0 = loC + chunk * ST_K, d1e = d0 + ST_K < hiC ? d0 + ST_K : hiC;
        int64_t pb = loB, i0 = loA;
        for (int64_t jj = d0; jj < d1e; ++jj) {
            const PairEnt ec = E[jj];
            const int64_t t3 = ec.t;
            int64_t lo = (t3 < LLONG_MIN + a.delta) ? LLONG_MIN : t3 - a.delta;
            lo = lo > wlo ? lo : wlo;
            pb = st_seek<true>(E, pb, hiB, t3);  // first middle not before t3
            if (pb == loB) continue;
            const int64_t tbl = E[pb - 1].t;  // the last middle before t3
            if (tbl <= lo) continue;
            i0 = st_seek<true>(E, i0, hiA, tbl);  // first edges strictly before it end at i0
            if (i0 == loA) continue;
            const uint32_t d3 = st_dir(ec, E[jj + 1], s_min_c);
            const int64_t cbt = E[pb].c0;
            cnt[0] += 1;
            if (d3) st_bwd_entry<CENSUS>(E, lane, t3, lo, i0, loA, pb, loB, cbt, s_min_a, y1_min, a.wfx, A1, cnt);
            else st_bwd_entry<CENSUS>(E, lane, t3, lo, i0, loA, pb, loB, cbt, s_min_a, y1_min, a.wfx, A0, cnt);
        }
        if constexpr (CENSUS) return;
        // set d3, slot 2 dm + d1 -> code 20 + 4 d1 + 2 dm + d3
        const int c0[4] = {20, 24, 22, 26}, c1[4] = {21, 25, 23, 27};
        if (a.kidx) {
            uint64_t *dst = a.win + (int64_t)a.kidx[u.jw] * 36 * 4;
            st_flush_global(A0, c0, dst, lane);
            st_flush_global(A1, c1, dst, lane);
        } else {
            st_flush(A0, c0, lds);
            st_flush(A1, c1, lds);
        }
    }
}

// CENSUS: out[0..2] += driver entries walked, 64-entry steps, valid lanes.
template <bool CENSUS>
__global__ void __launch_bounds__(ST_TPB) k_st_weight(DevGraph G, StArgs a) {
    __shared__ unsigned long long lds[36 * 4];
    for (int k = threadIdx.x; k < 36 * 4; k += ST_TPB) lds[k] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (TM_WAVE - 1);
    uint64_t cnt[3] = {0, 0, 0};
    while (true) {
        int64_t b = 0;
        if (lane == 0) b = (int64_t)atomicAdd(a.counter, 1ull);
        b = __shfl(b, 0, TM_WAVE);
        if (b >= a.ntask) break;
        st_task<CENSUS>(G, a, a.tasks[a.order[b]], lane, lds, cnt);
    }
    if constexpr (CENSUS) {
        if (lane == 0)
            for (int k = 0; k < 3; ++k) atomicAdd((unsigned long long *)&a.out[k], (unsigned long long)cnt[k]);
        return;
    }
    __syncthreads();
    for (int k = 20 * 4 + threadIdx.x; k < 28 * 4; k += ST_TPB) {
        const uint64_t v = lds[k];
        if (!v) continue;
        const int part = k & 3;
        uint64_t *o = a.out + (k & ~3);
        if (part == 0) tm_atomic_add_u128(o, o + 1, v, 0);
        else if (part == 1) atomicAdd((unsigned long long *)(o + 1), (unsigned long long)v);
        else if (part == 2) tm_atomic_add_u128(o + 2, o + 3, v, 0);
        else atomicAdd((unsigned long long *)(o + 3), (unsigned long long)v);
    }
}

// Per host thread, grow-only workspace of the per-call steps.
struct StWs {
    DevBuf cnt, units, tcnt, tasks, keys, vals, ctr, kflag, kept;
};
thread_local StWs t_st;

thread_local bool t_st_enabled = true;
// asked for a call's workspace bytes before it allocates them (nullptr: no
// limit, and the index is then also built on first use)
thread_local tm_st_grant_fn t_st_grant = nullptr;
thread_local void *t_st_grant_ctx = nullptr;

tm_status read_i64(const int64_t *d, int64_t *h, hipStream_t st) {
    TM_HIP(hipMemcpyAsync(h, d, 8, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    return TM_OK;
}

// The graph's static triangles, built on first use; false when there are too
// many candidates to check or triangles to keep (then the incidence-list
// sweep counts the triangles).
tm_status st_index(tm_graph *g, hipStream_t st, bool may_build, bool *ok) {
    std::lock_guard<std::mutex> lk(g_st_mu);
    *ok = false;
    if (g->st_state == 1) {
        *ok = true;
        return TM_OK;
    }
    if (g->st_state == 2 || !may_build) return TM_OK;
    const int64_t U = g->U, n = g->n;
    g->st_state = 2;
    if (U == 0 || n == 0) {
        g->st_ntri = 0;
        g->st_state = 1;
        *ok = true;
        return TM_OK;
    }
    DevBuf pab, deg, off, cur, onbr, opid, cnt, tot;
    TM_TRY(pab.alloc((size_t)U * 8));
    TM_TRY(deg.alloc((size_t)n * 4 + 16));
    TM_TRY(off.alloc((size_t)(n + 1) * 8));
    TM_TRY(cur.alloc((size_t)(n + 1) * 8));
    TM_TRY(onbr.alloc((size_t)U * 4));
    TM_TRY(opid.alloc((size_t)U * 4));
    TM_TRY(tot.alloc(16));
    const DevGraph G = dev_view(g);
    hipLaunchKernelGGL(k_st_zero, dim3(tm_blocks((n + 1) / 2 + 1, 256)), dim3(256), 0, st, deg.as<uint64_t>(),
                       (n + 1) / 2 + 1);
    hipLaunchKernelGGL(k_st_zero, dim3(tm_blocks(n + 1, 256)), dim3(256), 0, st, off.as<uint64_t>(), n + 1);
    hipLaunchKernelGGL(k_st_zero, dim3(1), dim3(64), 0, st, tot.as<uint64_t>(), (int64_t)2);
    hipLaunchKernelGGL(k_st_pair_ab, dim3(tm_blocks(g->ph_cap, 256)), dim3(256), 0, st, g->ph_slot.as<PairSlot>(),
                       g->ph_cap, pab.as<uint32_t>(), tot.as<unsigned long long>() + 1);
    hipLaunchKernelGGL(k_st_deg, dim3(tm_blocks(U, 256)), dim3(256), 0, st, pab.as<uint32_t>(), U,
                       deg.as<unsigned int>());
    hipLaunchKernelGGL(k_st_outdeg, dim3(tm_blocks(U, 256)), dim3(256), 0, st, pab.as<uint32_t>(), U,
                       deg.as<unsigned int>(), off.as<int64_t>());
    TM_HIP(hipGetLastError());
    TM_TRY(tm_scan_i64(off.as<int64_t>(), n, off.as<int64_t>() + n, st));
    TM_HIP(hipMemcpyAsync(cur.p, off.p, (size_t)(n + 1) * 8, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_st_outfill, dim3(tm_blocks(U, 256)), dim3(256), 0, st, pab.as<uint32_t>(), U,
                       deg.as<unsigned int>(), cur.as<int64_t>(), onbr.as<uint32_t>(), opid.as<int32_t>());
    hipLaunchKernelGGL(k_st_checks, dim3(tm_blocks(n, 256)), dim3(256), 0, st, off.as<int64_t>(), n,
                       tot.as<unsigned long long>());
    TM_HIP(hipGetLastError());
    int64_t checks[2] = {0, 0};  // candidate checks, largest pair
    TM_HIP(hipMemcpyAsync(checks, tot.p, 16, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    if ((uint64_t)checks[0] > ST_MAX_BUILD_CHECKS || (uint64_t)checks[0] > ST_CHECKS_PER_EDGE * (uint64_t)g->m_nl ||
        checks[1] >= ((int64_t)1 << 28))
        return TM_OK;
    TM_TRY(cnt.alloc((size_t)(U + 1) * 8));
    hipLaunchKernelGGL((k_st_tris<false>), dim3(tm_blocks(U, 256)), dim3(256), 0, st, G, off.as<int64_t>(), n, U,
                       onbr.as<uint32_t>(), opid.as<int32_t>(), cnt.as<int64_t>(), (StTri *)nullptr);
    TM_HIP(hipGetLastError());
    TM_TRY(tm_scan_i64(cnt.as<int64_t>(), U, cnt.as<int64_t>() + U, st));
    int64_t ntri = 0;
    TM_TRY(read_i64(cnt.as<int64_t>() + U, &ntri, st));
    size_t free_b = 0, total_b = 0;
    TM_HIP(hipMemGetInfo(&free_b, &total_b));
    if (ntri > INT32_MAX || ntri > g->m_nl || (double)ntri * sizeof(StTri) > (double)free_b / 8) return TM_OK;
    DevBuf tri;
    TM_TRY(tri.alloc((size_t)(ntri > 0 ? ntri : 1) * sizeof(StTri)));
    hipLaunchKernelGGL((k_st_tris<true>), dim3(tm_blocks(U, 256)), dim3(256), 0, st, G, off.as<int64_t>(), n, U,
                       onbr.as<uint32_t>(), opid.as<int32_t>(), cnt.as<int64_t>(), tri.as<StTri>());
    TM_HIP(hipGetLastError());
    TM_HIP(hipStreamSynchronize(st));
    g->st_tri.p = tri.p;
    g->st_tri.bytes = tri.bytes;
    g->st_tri.cap = tri.cap;
    tri.p = nullptr;
    tri.bytes = tri.cap = 0;
    g->device_bytes += (int64_t)g->st_tri.bytes;
    g->st_ntri = ntri;
    g->st_state = 1;
    *ok = true;
    return TM_OK;
}

}  // namespace

void tm_tri_static_enable(bool on) { t_st_enabled = on; }

void tm_tri_static_set_grant(tm_st_grant_fn fn, void *ctx) {
    t_st_grant = fn;
    t_st_grant_ctx = ctx;
}

tm_status tm_tri_static_prepare(tm_graph *g, hipStream_t st, bool *kept) {
    *kept = false;
    if (g->m_nl < ST_MIN_EDGES) return TM_OK;
    return st_index(g, st, true, kept);
}

bool tm_tri_static_kept(const tm_graph *g) {
    std::lock_guard<std::mutex> lk(g_st_mu);
    return g->st_state == 1 && g->m_nl >= ST_MIN_EDGES;
}

void tm_tri_static_release_thread_ws() {
    t_st.cnt.release();
    t_st.units.release();
    t_st.tcnt.release();
    t_st.tasks.release();
    t_st.keys.release();
    t_st.vals.release();
    t_st.ctr.release();
    t_st.kflag.release();
    t_st.kept.release();
}

namespace {

// The per-call set-up (units, tasks in claim order) and the launch: sums of
// codes 20..27 into out, or with census the work counts into out[0..2].
// *used = false when the path is off or the graph keeps no static triangles;
// nu, nt: units and tasks.
tm_status st_run(const tm_graph *gc, int64_t delta, int64_t s, int64_t L, uint64_t seed, double p,
                 const int32_t *kidx, const uint64_t *wfx, uint64_t *out, uint64_t *win, hipStream_t st,
                 uint64_t pass, int groups_per_cu, bool census, bool *used, int64_t *nu_out, int64_t *nt_out) {
    *used = false;
    *nu_out = *nt_out = 0;
    if (L <= 0) return TM_OK;
    tm_graph *g = const_cast<tm_graph *>(gc);  // the index is a cache of the immutable graph
    const tm_st_grant_fn grant = census ? nullptr : t_st_grant;
    auto fits = [&](int64_t bytes) { return !grant || grant(t_st_grant_ctx, bytes); };
    bool ok = false;
    TM_TRY(st_index(g, st, grant == nullptr, &ok));
    if (!ok) return TM_OK;
    const int64_t ntri = g->st_ntri;
    if (ntri == 0) {
        *used = true;
        return TM_OK;
    }
    // the kept window ids, when their list is small enough to build per call
    const int64_t J = (g->t_span - s) / L + 1;
    // with a grant hook, the path is left to the incidence-list sweep as soon
    // as the hook refuses its workspace (counts, window list, scans, units,
    // tasks, sort)
    int64_t ws = (ntri + 1) * 8 + (J <= ST_MAX_WINDOW_LIST ? (2 * J + 1) * 8 : 0) +
                 tm_scan_ws_bytes(ntri > J ? ntri : J);
    if (!fits(ws)) return TM_OK;
    *used = true;
    const DevGraph G = dev_view(g);
    const StTri *tris = g->st_tri.as<StTri>();
    StWs &W = t_st;
    void *tok = census ? nullptr : tm_prof_begin("tri_static_prep", st, pass);
    TM_TRY(W.cnt.reserve((size_t)(ntri + 1) * 8));
    const int64_t *kept = nullptr, *nkept = nullptr;
    if (J <= ST_MAX_WINDOW_LIST) {
        TM_TRY(W.kflag.reserve((size_t)(J + 1) * 8));
        TM_TRY(W.kept.reserve((size_t)J * 8));
        hipLaunchKernelGGL(k_st_kept_flags, dim3(tm_blocks(J, 256)), dim3(256), 0, st, J, kidx, seed, p,
                           W.kflag.as<int64_t>());
        TM_HIP(hipGetLastError());
        TM_TRY(tm_scan_i64(W.kflag.as<int64_t>(), J, W.kflag.as<int64_t>() + J, st));
        hipLaunchKernelGGL(k_st_kept_fill, dim3(tm_blocks(J, 256)), dim3(256), 0, st, J, kidx, seed, p,
                           W.kflag.as<int64_t>(), W.kept.as<int64_t>());
        TM_HIP(hipGetLastError());
        kept = W.kept.as<int64_t>();
        nkept = W.kflag.as<int64_t>() + J;
    }
    hipLaunchKernelGGL((k_st_units<false>), dim3(tm_blocks(ntri, 256)), dim3(256), 0, st, G, tris, ntri, s, L, seed,
                       p, kidx, kept, nkept, W.cnt.as<int64_t>(), (StUnit *)nullptr, (int64_t *)nullptr);
    TM_HIP(hipGetLastError());
    TM_TRY(tm_scan_i64(W.cnt.as<int64_t>(), ntri, W.cnt.as<int64_t>() + ntri, st));
    int64_t nu = 0;
    TM_TRY(read_i64(W.cnt.as<int64_t>() + ntri, &nu, st));
    if (nu == 0) {
        tm_prof_end(tok, st);
        return TM_OK;
    }
    if (nu > UINT32_MAX) return TM_ENOMEM;
    ws += (int64_t)nu * (int64_t)(sizeof(StUnit) + 8) + 8 + tm_scan_ws_bytes(nu);
    if (!fits(ws)) {
        tm_prof_end(tok, st);
        *used = false;
        return TM_OK;
    }
    TM_TRY(W.units.reserve((size_t)nu * sizeof(StUnit)));
    TM_TRY(W.tcnt.reserve((size_t)(nu + 1) * 8));
    hipLaunchKernelGGL((k_st_units<true>), dim3(tm_blocks(ntri, 256)), dim3(256), 0, st, G, tris, ntri, s, L, seed,
                       p, kidx, kept, nkept, W.cnt.as<int64_t>(), W.units.as<StUnit>(), W.tcnt.as<int64_t>());
    TM_HIP(hipGetLastError());
    TM_TRY(tm_scan_i64(W.tcnt.as<int64_t>(), nu, W.tcnt.as<int64_t>() + nu, st));
    int64_t nt = 0;
    TM_TRY(read_i64(W.tcnt.as<int64_t>() + nu, &nt, st));
    if (nt > UINT32_MAX) return TM_ENOMEM;
    ws += nt * 20 + 8 + tm_radix_sort_bytes(nt);
    if (!fits(ws)) {
        tm_prof_end(tok, st);
        *used = false;
        return TM_OK;
    }
    *nu_out = nu;
    *nt_out = nt;
    TM_TRY(W.tasks.reserve((size_t)nt * 8));
    TM_TRY(W.keys.reserve((size_t)nt * 8));
    TM_TRY(W.vals.reserve((size_t)nt * 4));
    TM_TRY(W.ctr.reserve(8));
    hipLaunchKernelGGL(k_st_tasks, dim3(tm_blocks(nu, 256)), dim3(256), 0, st, W.units.as<StUnit>(), nu,
                       W.tcnt.as<int64_t>(), delta, L, W.tasks.as<uint64_t>(), W.keys.as<uint64_t>(),
                       W.vals.as<uint32_t>());
    hipLaunchKernelGGL(k_st_zero, dim3(1), dim3(64), 0, st, W.ctr.as<uint64_t>(), (int64_t)1);
    TM_HIP(hipGetLastError());
    TM_TRY(tm_radix_sort(W.keys.as<uint64_t>(), W.vals.as<uint32_t>(), nt, 32, st));
    tm_prof_end(tok, st);
    StArgs a;
    a.delta = delta;
    a.s = s;
    a.L = L;
    a.wfx = wfx;
    a.tris = tris;
    a.units = W.units.as<StUnit>();
    a.tasks = W.tasks.as<uint64_t>();
    a.order = W.vals.as<uint32_t>();
    a.ntask = nt;
    a.counter = W.ctr.as<unsigned long long>();
    a.out = out;
    a.kidx = kidx;
    a.win = win;
    int dev = g->device, ncu = 0;
    TM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu <= 0) ncu = 256;
    int64_t nb = (nt + ST_TPB / TM_WAVE - 1) / (ST_TPB / TM_WAVE);  // one task per wave
    if (nb > (int64_t)ncu * groups_per_cu) nb = (int64_t)ncu * groups_per_cu;
    if (nb < 1) nb = 1;
    if (census) {
        hipLaunchKernelGGL((k_st_weight<true>), dim3((unsigned)nb), dim3(ST_TPB), 0, st, G, a);
        return tm_hip_status(hipGetLastError());
    }
    void *tk = tm_prof_begin("tri_static_weight", st, pass);
    hipLaunchKernelGGL((k_st_weight<false>), dim3((unsigned)nb), dim3(ST_TPB), 0, st, G, a);
    TM_HIP(hipGetLastError());
    tm_prof_end(tk, st);
    return TM_OK;
}

}  // namespace

tm_status tm_tri_static_weight(const tm_graph *gc, int64_t delta, int64_t s, int64_t L, uint64_t seed, double p,
                               const int32_t *kidx, const uint64_t *wfx, uint64_t *out, uint64_t *win,
                               hipStream_t st, uint64_t pass, bool shared, bool *used) {
    *used = false;
    if (!t_st_enabled) return TM_OK;
    // TM_TRI_STATIC=0 keeps the incidence-list sweep, =1 takes this path on
    // any graph; otherwise graphs below ST_MIN_EDGES keep the list sweep,
    // whose whole pass there is shorter than this path's set-up
    const char *e = getenv("TM_TRI_STATIC");
    if (e && e[0] == '0') return TM_OK;
    if (!(e && e[0] == '1') && gc->m_nl < ST_MIN_EDGES) return TM_OK;
    // Beside the pass's other kernels two work-groups per CU (eight waves,
    // two per SIMD at 122 VGPRs) leave each SIMD room for one wave of the
    // 2-node/star sweep and one of the backward star sweep: on a 10M-edge Zipf
    // graph (100k nodes) four estimate passes took 109 ms against 136 ms with
    // three work-groups per CU and 141 ms with eight.  Alone, eight fill the
    // CUs (c 30, p 0.1: 26 ms against 38 ms with two).
    int64_t nu, nt;
    return st_run(gc, delta, s, L, seed, p, kidx, wfx, out, win, st, pass, shared ? 2 : 8, false, used, &nu, &nt);
}

tm_status tm_tri_static_census_impl(const tm_graph *g, int64_t delta, int64_t s, int64_t L, uint64_t seed, double p,
                                    tm_tri_census *c, hipStream_t st) {
    DevBuf o;
    TM_TRY(o.alloc(32));
    hipLaunchKernelGGL(k_st_zero, dim3(1), dim3(64), 0, st, o.as<uint64_t>(), (int64_t)4);
    TM_HIP(hipGetLastError());
    bool used = false;
    int64_t nu = 0, nt = 0;
    TM_TRY(st_run(g, delta, s, L, seed, p, nullptr, nullptr, o.as<uint64_t>(), nullptr, st, 0, 8, true, &used, &nu,
                  &nt));
    if (!used) return TM_EUNSUPPORTED;
    uint64_t h[4];
    TM_HIP(hipMemcpyAsync(h, o.p, 32, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    c->triangles = g->st_ntri;
    c->units = nu;
    c->tasks = nt;
    c->drivers = (int64_t)h[0];
    c->steps = (int64_t)h[1];
    c->combos = (int64_t)h[2];
    return TM_OK;
}
