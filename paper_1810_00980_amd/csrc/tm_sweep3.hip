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

namespace {

constexpr int SW_TPB = 256;
constexpr int SW_WAVES = SW_TPB / TM_WAVE;

enum : int { MODE_COUNT = 0, MODE_WEIGHT = 1, MODE_HIST = 2 };

struct SweepArgs {
    int64_t delta;
    // windows (estimate): anchor kept when its window's draw is below p
    int32_t windowed;      // 0 none, 1 kept windows of (s, L, seed, p), 2 one window [s, L]
    int64_t s, L;
    uint64_t seed;
    double p;
    const uint64_t *wfx;   // delta+1 fixed-point weights (MODE_WEIGHT)
    uint64_t *hist;        // 36 x (delta+1) x {lo, hi} (MODE_HIST)
    uint64_t *out;         // 36 x {count lo, count hi, weight lo, weight hi}
    int64_t *counter;      // work queue head
    uint32_t want_fwd;     // bit mask: 1 two-node, 2 star B, 4 star A, 8 triangle
    int64_t n_entries;
};

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

// number of entries of directed pair p with time < t
__device__ inline int64_t pair_before(const DevGraph &G, int32_t p, int64_t t) {
    int64_t t0 = G.pb_tfirst[p];
    if (t <= t0) return 0;
    int shift = G.pb_meta[2 * p];
    int64_t nb = G.pb_meta[2 * p + 1];
    int64_t b = (t - t0) >> shift;
    int64_t base = G.sp_beg[p];
    if (b >= nb) return G.sp_beg[p + 1] - base;
    const int32_t *bi = G.pb_idx + G.pb_off[p];
    int64_t lo = bi[b], hi = bi[b + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (G.pr_t[base + mid] < t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// directed pair ids (u -> v, v -> u) of the unordered pair {u, v}; -1 if absent
__device__ inline void pair_ids(const DevGraph &G, uint32_t u, uint32_t v, int32_t *puv, int32_t *pvu) {
    uint32_t a = u < v ? u : v, b = u < v ? v : u;
    uint64_t key = ((uint64_t)a << 32) | b;
    int64_t cap = G.ph_cap;
    uint64_t h = tm_pair_hash(key, cap);
    *puv = -1;
    *pvu = -1;
    for (int64_t probe = 0; probe < cap; ++probe) {
        uint64_t k = G.ph_key[h];
        if (k == key) {
            int32_t f = G.ph_val[2 * h], r = G.ph_val[2 * h + 1];  // a -> b, b -> a
            *puv = u < v ? f : r;
            *pvu = u < v ? r : f;
            return;
        }
        if (k == ~0ull) return;
        h = (h + 1) & (uint64_t)(cap - 1);
    }
}

// entries of pair p with tlo < t < thi
__device__ inline uint64_t pair_between_id(const DevGraph &G, int32_t p, int64_t tlo, int64_t thi) {
    if (p < 0) return 0;
    return (uint64_t)(pair_before(G, p, thi) - pair_before(G, p, tlo + 1));
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

template <int MODE, int NC>
__device__ inline void flush(const Acc<MODE, NC> &A, const int *codes, unsigned long long *lds) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        int code = codes[k];
        if (code < 0) continue;
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

// forward sweep of one anchor (codes 0..27)
template <int MODE>
__device__ inline void sweep_fwd(const DevGraph &G, const SweepArgs &a, int64_t i, int64_t end, uint32_t y1,
                                 uint32_t d1, int64_t t1, int64_t hi, unsigned long long *lds) {
    // slots: 0..3 two-node [2*d2+d3], 4..7 star B, 8..11 star A, 12..15 triangle
    Acc<MODE, 16> A;
    A.clear();
    const bool two = (a.want_fwd & 1u) && d1 == 0;
    const bool sb = a.want_fwd & 2u, sa = a.want_fwd & 4u, tri = a.want_fwd & 8u;
    uint64_t cs0 = 0, cs1 = 0, ca0 = 0, ca1 = 0;  // middles before the current time group
    uint64_t ps0 = 0, ps1 = 0, pa0 = 0, pa1 = 0;  // entries of the current time group
    int64_t tg = t1;
    for (int64_t j = i + 1; j < end; ++j) {
        int64_t tj = G.inc_t[j];
        if (tj > hi) break;
        if (tj == t1) continue;
        if (tj != tg) {
            cs0 += ps0; cs1 += ps1; ca0 += pa0; ca1 += pa1;
            ps0 = ps1 = pa0 = pa1 = 0;
            tg = tj;
        }
        uint32_t nd = G.inc_nd[j];
        uint32_t yj = nd & 0x7FFFFFFFu, dj = nd >> 31;
        int64_t dlt = tj - t1;
        uint64_t w = 0;
        if constexpr (MODE == MODE_WEIGHT) w = weight_of<MODE>(a, dlt);
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
                int32_t p01, p10;
                pair_ids(G, y1, yj, &p01, &p10);
                uint64_t c01 = pair_between_id(G, p01, t1, tj);
                uint64_t c10 = pair_between_id(G, p10, t1, tj);
                acc_add<MODE, 16>(A, 12, dj, c01, w, a.hist, 20 + 4 * (int)d1, dlt, a.delta);
                acc_add<MODE, 16>(A, 14, dj, c10, w, a.hist, 22 + 4 * (int)d1, dlt, a.delta);
            }
        }
        if (dj) ++pa1; else ++pa0;
    }
    int codes[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        codes[k] = two ? k : -1;
        codes[4 + k] = 4 + 4 * (int)d1 + k;
        codes[8 + k] = 12 + 4 * (int)d1 + k;
        codes[12 + k] = 20 + 4 * (int)d1 + k;
    }
    flush<MODE, 16>(A, codes, lds);
}

// backward sweep of one anchor (codes 28..35): star with e2 on e3's pair
template <int MODE>
__device__ inline void sweep_bwd(const DevGraph &G, const SweepArgs &a, int64_t jj, int64_t beg, uint32_t y3,
                                 uint32_t d3, int64_t t3, int64_t lo, unsigned long long *lds) {
    // slots [2*d1 + d2]: v is added at slot (2*d1 + d2), d1 runtime -> use base 2*d2 with dsel = d1
    Acc<MODE, 4> A;  // slot index: d2 * 2 + d1
    A.clear();
    uint64_t cs0 = 0, cs1 = 0, ps0 = 0, ps1 = 0;
    int64_t tg = t3;
    for (int64_t i = jj - 1; i >= beg; --i) {
        int64_t ti = G.inc_t[i];
        if (ti < lo) break;
        if (ti == t3) continue;
        if (ti != tg) {
            cs0 += ps0; cs1 += ps1;
            ps0 = ps1 = 0;
            tg = ti;
        }
        uint32_t nd = G.inc_nd[i];
        uint32_t yi = nd & 0x7FFFFFFFu, di = nd >> 31;
        if (yi != y3) {
            int64_t dlt = t3 - ti;
            uint64_t w = 0;
            if constexpr (MODE == MODE_WEIGHT) w = weight_of<MODE>(a, dlt);
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
    }
    int codes[4];
    // slot (2*d2 + d1) -> code 28 + 4*d1 + 2*d2 + d3
    codes[0] = 28 + 0 + 0 + (int)d3;  // d2=0,d1=0
    codes[1] = 28 + 4 + 0 + (int)d3;  // d2=0,d1=1
    codes[2] = 28 + 0 + 2 + (int)d3;  // d2=1,d1=0
    codes[3] = 28 + 4 + 2 + (int)d3;  // d2=1,d1=1
    flush<MODE, 4>(A, codes, lds);
}

template <int MODE, bool FWD>
__global__ void __launch_bounds__(SW_TPB) k_sweep3(DevGraph G, SweepArgs a) {
    __shared__ unsigned long long lds[36 * 4];
    for (int k = threadIdx.x; k < 36 * 4; k += SW_TPB) lds[k] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (TM_WAVE - 1);
    const int64_t nE = a.n_entries;
    while (true) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd((unsigned long long *)a.counter, (unsigned long long)TM_WAVE);
        base = __shfl(base, 0, TM_WAVE);
        if (base >= nE) break;
        int64_t i = base + lane;
        if (i < nE) {
            int64_t x = owner_of(G.inc_off, G.n, i);
            int64_t lb = G.inc_off[x], le = G.inc_off[x + 1];
            uint32_t nd = G.inc_nd[i];
            uint32_t y = nd & 0x7FFFFFFFu, d = nd >> 31;
            int64_t t = G.inc_t[i];
            bool go = true;
            int64_t wlo = LLONG_MIN, whi = LLONG_MAX;
            if (a.windowed == 1) {
                int64_t j = (t - a.s) / a.L + 1;
                go = keep_window(a.seed, (uint64_t)j, a.p);
                wlo = a.s + (j - 1) * a.L;
                whi = a.s + j * a.L - 1;
            } else if (a.windowed == 2) {
                wlo = a.s;
                whi = a.L;
                go = t >= wlo && t <= whi;
            }
            if (go) {
                if (FWD) {
                    int64_t hi = (t > LLONG_MAX - a.delta) ? LLONG_MAX : t + a.delta;
                    hi = hi < whi ? hi : whi;
                    sweep_fwd<MODE>(G, a, i, le, y, d, t, hi, lds);
                } else {
                    int64_t lo = (t < LLONG_MIN + a.delta) ? LLONG_MIN : t - a.delta;
                    lo = lo > wlo ? lo : wlo;
                    sweep_bwd<MODE>(G, a, i, lb, y, d, t, lo, lds);
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

template <int MODE>
tm_status launch_pair(const tm_graph *g, SweepArgs a, bool fwd, bool bwd, hipStream_t st) {
    DevGraph G = dev_view(g);
    int dev = g->device, ncu = 0;
    TM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu <= 0) ncu = 256;
    int64_t nE = a.n_entries;
    int64_t want_blocks = (nE + SW_TPB - 1) / SW_TPB;
    int64_t nb = (int64_t)ncu * 8;
    if (nb > want_blocks) nb = want_blocks;
    if (nb < 1) nb = 1;
    static const char *names[3][2] = {{"sweep3_fwd_count", "sweep3_bwd_count"},
                                      {"sweep3_fwd_weight", "sweep3_bwd_weight"},
                                      {"sweep3_fwd_hist", "sweep3_bwd_hist"}};
    if (fwd) {
        TM_HIP(hipMemsetAsync(a.counter, 0, 8, st));
        void *tok = tm_prof_begin(names[MODE][0], st);
        hipLaunchKernelGGL((k_sweep3<MODE, true>), dim3((unsigned)nb), dim3(SW_TPB), 0, st, G, a);
        TM_HIP(hipGetLastError());
        tm_prof_end(tok, st);
    }
    if (bwd) {
        TM_HIP(hipMemsetAsync(a.counter + 1, 0, 8, st));
        SweepArgs b = a;
        b.counter = a.counter + 1;
        void *tok = tm_prof_begin(names[MODE][1], st);
        hipLaunchKernelGGL((k_sweep3<MODE, false>), dim3((unsigned)nb), dim3(SW_TPB), 0, st, G, b);
        TM_HIP(hipGetLastError());
        tm_prof_end(tok, st);
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

}  // namespace

tm_status tm_sweep_census_impl(const tm_graph *g, int64_t delta, int64_t *fwd, int64_t *bwd, hipStream_t st) {
    DevBuf o;
    TM_TRY(o.alloc(64));
    TM_HIP(hipMemsetAsync(o.p, 0, 16, st));
    if (g->m_nl > 0) {
        unsigned nb = tm_blocks(2 * g->m_nl, SW_TPB);
        if (nb > 8192) nb = 8192;
        hipLaunchKernelGGL(k_census, dim3(nb), dim3(SW_TPB), 0, st, dev_view(g), delta, o.as<unsigned long long>());
        TM_HIP(hipGetLastError());
    }
    int64_t h[2];
    TM_HIP(hipMemcpyAsync(h, o.p, 16, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    *fwd = h[0];
    *bwd = h[1];
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

// mode: 0 counts, 1 counts + weights (needs L), 2 counts + histograms.
// out_dev: 36 x 4 u64 (count lo/hi, weight lo/hi), zeroed here.
// hist_dev: 36 x (delta+1) x 2 u64 (mode 2), zeroed here.
tm_status tm_sweep3(const tm_graph *g, uint64_t code_mask_lo, int mode, int64_t delta, int windowed, int64_t s,
                    int64_t L, uint64_t seed, double p, uint64_t *out_dev, uint64_t *hist_dev, uint64_t *wfx_dev,
                    int64_t *counter_dev, hipStream_t st) {
    SweepArgs a;
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
    uint32_t wf = 0;
    if (code_mask_lo & 0xFull) wf |= 1;
    if (code_mask_lo & 0xFF0ull) wf |= 2;
    if (code_mask_lo & 0xFF000ull) wf |= 4;
    if (code_mask_lo & 0xFF00000ull) wf |= 8;
    bool bwd = (code_mask_lo >> 28) & 0xFFull;
    a.want_fwd = wf;
    TM_HIP(hipMemsetAsync(out_dev, 0, 36 * 4 * 8, st));
    if (mode == MODE_HIST) TM_HIP(hipMemsetAsync(hist_dev, 0, (size_t)36 * (delta + 1) * 16, st));
    if (mode == MODE_WEIGHT) {
        hipLaunchKernelGGL(k_weights_fx, dim3(tm_blocks(delta + 1, 256)), dim3(256), 0, st, delta, L, wfx_dev);
        TM_HIP(hipGetLastError());
    }
    if (a.n_entries == 0) return TM_OK;
    switch (mode) {
        case MODE_COUNT: return launch_pair<MODE_COUNT>(g, a, wf != 0, bwd, st);
        case MODE_WEIGHT: return launch_pair<MODE_WEIGHT>(g, a, wf != 0, bwd, st);
        default: return launch_pair<MODE_HIST>(g, a, wf != 0, bwd, st);
    }
}
