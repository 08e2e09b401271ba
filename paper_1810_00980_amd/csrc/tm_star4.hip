// Four-edge stars whose first two edges join the center to the same leaf:
// (x, a), (x, a), (x, b), (x, c) with a, b, c distinct and each edge's
// direction fixed by the motif, e.g. the star of the paper's Fig. 1,
// (0,1),(0,1),(0,2),(0,3) (Sec. 2, Definitions "temporal motif" and "motif
// delta-instance"; the k-temporal star of Sec. 3).
//
// Every instance lies in the time-sorted incidence list of its center x.
// For an anchor e1 (entry i of x's list, leaf a) and a later entry e4 of
// x's list (leaf c), the instances with first edge e1 and last edge e4 all
// have the duration t4 - t1, and their number is a count of middles:
//
//   mid(e1, e4) = sum over e3 (leaf b != a, c; t1 < t3 < t4) of A(t3),
//   A(t) = number of second edges e2 (leaf a, t1 < t2 < t).
//
// One forward scan of x's list from e1 keeps A, S = the sum of A(t3) over
// the third edges seen so far (leaf != a), and T_c = the same sum restricted
// to leaf c, so that mid(e1, e4) = S - T_c.  T_c is kept in LDS for the
// node's K heaviest leaves (most edges on the pair); for any other leaf c it
// is computed when e4 needs it, from the pair timelines: the third edges on
// the pair {x, c} between t1 and t4, each with A from a lookup in the pair
// {x, a}.  Entries tied in time are taken as a group: the group's last edges
// use the sums of earlier groups only, then the group's second and third
// edges join them, so tied edges never share an instance.
//
// The whole duration histogram is never built for an estimate: each (e1, e4)
// adds its count times the fixed-point weight round(2^52 L / (L - Delta)) to
// an exact 128-bit sum (Algorithm 1's weighting, summed in integers).
#include "tm_common.h"

#include <limits.h>

#include <mutex>

#include "tm_sweep_dev.h"

namespace {

using namespace sweepdev;

constexpr int S4_TPB = 128;             // lanes per work-group (K 64-bit sums each in LDS)
constexpr int S4_K = 32;                // heavy leaves per node
constexpr uint8_t S4_LIGHT = 0xFF;      // rank of a leaf outside its node's heaviest K

struct Star4Args {
    int64_t delta;
    int32_t windowed;   // 0: every anchor; 1: anchors in windows kept by (s, L, seed, p); 2: window [s, L]
    int64_t s, L;
    uint64_t seed;
    double p;
    uint32_t d[4];        // direction of each motif edge at the center (0: leaves it, 1: enters it)
    const uint64_t *wfx;  // delta + 1 fixed-point weights (MODE_WEIGHT)
    uint64_t *hist;       // delta + 1 bins {lo, hi} (MODE_HIST)
    uint64_t *out;        // count lo, count hi, weight lo, weight hi
    unsigned long long *counter;
    const uint8_t *rank;  // heavy rank of each incidence entry's other endpoint at the list's owner
    int64_t n_entries;
};

// which count of a pair timeline {min, max} is direction d at node x:
// c[0] counts min -> max edges, c[1] max -> min
__device__ inline int dir_index(uint32_t x, uint32_t y, uint32_t d) { return (x < y) ? (int)d : 1 - (int)d; }

// T_c of a leaf outside the heavy set: sum over the entries of the pair
// {x, c} with direction d3 and time in (t1, t4) of A(t) = (direction-d2
// entries of the pair {x, a} before t) - base2
__device__ inline uint64_t light_sum(const DevGraph &G, uint32_t x, uint32_t c, uint32_t d3, int64_t t1, int64_t t4,
                                    const PairView &pa, int sel2, int64_t base2) {
    PairView pc;
    if (pair_find(G, x, c, pc) < 0) return 0;
    int64_t cc[2];
    pc.le(G, t1, cc);
    const int64_t lo = cc[0] + cc[1];
    pc.lt(G, t4, cc);
    const int64_t hi = cc[0] + cc[1];
    const bool x_min = x < c;
    uint64_t sum = 0;
    int64_t c0 = lo < hi ? pc.en[lo].c0 : 0;
    for (int64_t e = lo; e < hi; ++e) {
        const PairEnt q = pc.en[e];
        const int64_t c1 = pc.en[e + 1].c0;  // the entry after (at worst the sentinel)
        const bool min_to_max = c1 - c0 == 1;
        c0 = c1;
        const uint32_t dx = x_min ? (min_to_max ? 0u : 1u) : (min_to_max ? 1u : 0u);
        if (dx != d3) continue;
        int64_t ca[2];
        pa.lt(G, q.t, ca);
        sum += (uint64_t)(ca[sel2] - base2);
    }
    return sum;
}

__device__ inline void wave_add_u128(uint64_t &lo, uint64_t &hi) {
#pragma unroll
    for (int o = TM_WAVE / 2; o > 0; o >>= 1) {
        const uint64_t olo = __shfl_xor(lo, o, TM_WAVE);
        const uint64_t ohi = __shfl_xor(hi, o, TM_WAVE);
        tm_add_u128(lo, hi, olo, ohi);
    }
}

template <int MODE>
__global__ void __launch_bounds__(S4_TPB) k_star4(DevGraph G, Star4Args a) {
    __shared__ unsigned long long T[S4_K][S4_TPB];  // per lane: T_c of the node's heavy leaves
    const int tid = threadIdx.x, lane = tid & (TM_WAVE - 1);
    uint64_t cl = 0, ch = 0, wl = 0, wh = 0;  // this lane's sums
    const int64_t nE = a.n_entries;
    while (true) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd(a.counter, (unsigned long long)TM_WAVE);
        base = __shfl(base, 0, TM_WAVE);
        if (base >= nE) break;
        const int64_t i = base + lane;
        if (i >= nE) continue;
        const uint32_t nd1 = G.inc_nd[i];
        if ((nd1 >> 31) != a.d[0]) continue;
        const uint32_t y1 = nd1 & 0x7FFFFFFFu;
        const int64_t t1 = G.inc_t[i];
        int64_t whi = LLONG_MAX;
        if (a.windowed == 1) {
            const int64_t jw = (t1 - a.s) / a.L + 1;
            if (!keep_window(a.seed, (uint64_t)jw, a.p)) continue;
            whi = a.s + jw * a.L - 1;
        } else if (a.windowed == 2) {
            if (t1 < a.s || t1 > a.L) continue;
            whi = a.L;
        }
        int64_t hi = (t1 > LLONG_MAX - a.delta) ? LLONG_MAX : t1 + a.delta;
        hi = hi < whi ? hi : whi;
        const uint32_t x = (uint32_t)owner_of(G.inc_off, G.n, i);
        // second edges on the pair {x, a}: none in (t1, hi] means no instance
        PairView pa;
        if (pair_find(G, x, y1, pa) < 0) continue;
        const int sel2 = dir_index(x, y1, a.d[1]);
        int64_t cc[2];
        pa.le(G, t1, cc);
        const int64_t base2 = cc[sel2];
        pa.le(G, hi, cc);
        if (cc[sel2] == base2) continue;
        for (int k = 0; k < S4_K; ++k) T[k][tid] = 0;
        uint64_t A = 0, S = 0;
        const int64_t le = G.inc_off[x + 1];
        int64_t j = i + 1;
        while (j < le && G.inc_t[j] == t1) ++j;  // ties with the anchor
        // The last-edge role of an entry e4 (direction d3, leaf c != a) adds
        // S - T_c, then its second-edge (leaf a, direction d2: A += 1) or
        // third-edge role (leaf != a, direction d3: S += A, T_c += A) joins
        // the sums.  An entry whose time no neighbour shares does both at
        // once; a group of entries tied in time takes the last-edge roles of
        // all its entries first and their other roles after (star_group), so
        // that tied edges never share an instance.  Entries are read four at
        // a time, with the next chunk's first time for the tie test.
        auto last_edge = [&](int64_t tq, uint32_t nd, uint8_t r, uint64_t w) {
            const uint32_t c = nd & 0x7FFFFFFFu;
            if ((nd >> 31) != a.d[3] || c == y1) return;
            const uint64_t tc = r != S4_LIGHT ? (uint64_t)T[r][tid]
                                               : light_sum(G, x, c, a.d[2], t1, tq, pa, sel2, base2);
            const uint64_t cnt = S - tc;
            if (!cnt) return;
            tm_add_u128(cl, ch, cnt, 0);
            if constexpr (MODE == MODE_WEIGHT) tm_add_u128(wl, wh, cnt * w, __umul64hi(cnt, w));
            if constexpr (MODE == MODE_HIST) {
                uint64_t *h = a.hist + 2 * (tq - t1);
                tm_atomic_add_u128(h, h + 1, cnt, 0);
            }
        };
        while (j < le) {
            int64_t tq[4];
            uint32_t nq[4];
            uint8_t rq[4];
            uint64_t wq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t k = j + u < le ? j + u : le - 1;
                tq[u] = j + u < le ? G.inc_t[k] : LLONG_MAX;
                nq[u] = G.inc_nd[k];
                rq[u] = a.rank[k];
            }
            const int64_t tn = j + 4 < le ? G.inc_t[j + 4] : LLONG_MAX;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                wq[u] = 0;
                if constexpr (MODE == MODE_WEIGHT) {
                    if (tq[u] <= hi) wq[u] = a.wfx[tq[u] - t1];
                }
            }
            int64_t jn = j + 4;
            bool stop = false;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (stop) continue;
                if (j + u >= le || tq[u] > hi) {
                    stop = true;
                    jn = le;
                    continue;
                }
                const int64_t tnext = u < 3 ? tq[u + 1] : tn;
                if (tq[u] == tnext) {
                    // a group of tied entries from j + u
                    const int64_t tg = tq[u];
                    int64_t ge = j + u + 1;
                    while (ge < le && G.inc_t[ge] == tg) ++ge;
                    if (S) {
                        for (int64_t q = j + u; q < ge; ++q) last_edge(tg, G.inc_nd[q], a.rank[q], wq[u]);
                    }
                    uint64_t addA = 0;
                    for (int64_t q = j + u; q < ge; ++q) {
                        const uint32_t nd = G.inc_nd[q];
                        const uint32_t y = nd & 0x7FFFFFFFu, dq = nd >> 31;
                        if (y == y1) {
                            addA += dq == a.d[1];
                        } else if (dq == a.d[2] && A) {
                            S += A;
                            const uint8_t r = a.rank[q];
                            if (r != S4_LIGHT) T[r][tid] += A;
                        }
                    }
                    A += addA;
                    jn = ge;
                    stop = true;
                    continue;
                }
                if (S) last_edge(tq[u], nq[u], rq[u], wq[u]);
                const uint32_t y = nq[u] & 0x7FFFFFFFu, dq = nq[u] >> 31;
                if (y == y1) {
                    A += dq == a.d[1];
                } else if (dq == a.d[2] && A) {
                    S += A;
                    if (rq[u] != S4_LIGHT) T[rq[u]][tid] += A;
                }
            }
            j = jn;
        }
    }
    wave_add_u128(cl, ch);
    if constexpr (MODE == MODE_WEIGHT) wave_add_u128(wl, wh);
    if (lane == 0) {
        if (cl | ch) tm_atomic_add_u128(a.out, a.out + 1, cl, ch);
        if (wl | wh) tm_atomic_add_u128(a.out + 2, a.out + 3, wl, wh);
    }
}

// --------------------------------------------------------- heavy leaves

// two records per unordered pair {u, v} of n edges: (u, n) -> v and (v, n) -> u,
// keyed by node and then by decreasing n
__global__ void k_s4_records(const PairSlot *slot, int64_t cap, unsigned long long *cnt, uint64_t *keys,
                             uint32_t *vals) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= cap) return;
    const PairSlot s = slot[h];
    if (s.id < 0) return;
    const uint32_t u = (uint32_t)(s.key >> 32), v = (uint32_t)s.key;
    const uint64_t inv = 0xFFFFFFFFull - (uint64_t)s.n;
    const unsigned long long k = atomicAdd(cnt, 2ull);
    keys[k] = ((uint64_t)u << 32) | inv;
    vals[k] = v;
    keys[k + 1] = ((uint64_t)v << 32) | inv;
    vals[k + 1] = u;
}

// beg[x] = first record of node x, len[x] = its records (nodes without any: 0)
__global__ void k_s4_segments(const uint64_t *keys, int64_t nr, int64_t *beg, int64_t *len) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const uint64_t x = keys[r] >> 32;
    if (r == 0 || (keys[r - 1] >> 32) != x) beg[x] = r;
    if (r == nr - 1 || (keys[r + 1] >> 32) != x) len[x] = r + 1;  // end, made a length below
}

__global__ void k_s4_lengths(const int64_t *beg, int64_t *len, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n && len[x] > 0) len[x] -= beg[x];
}

// per incidence entry: the rank of its other endpoint among its owner's K
// heaviest neighbours, or S4_LIGHT
__global__ void k_s4_rank(DevGraph G, const uint32_t *vals, const int64_t *beg, const int64_t *len, uint8_t *rank) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 2 * G.m_nl) return;
    const int64_t x = owner_of(G.inc_off, G.n, q);
    const uint32_t y = G.inc_nd[q] & 0x7FFFFFFFu;
    const int64_t b = beg[x], k = len[x] < S4_K ? len[x] : S4_K;
    uint8_t r = S4_LIGHT;
    for (int64_t s = 0; s < k; ++s)
        if (vals[b + s] == y) r = (uint8_t)s;
    rank[q] = r;
}

__global__ void k_s4_zero(uint64_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_s4_weights(int64_t delta, int64_t L, uint64_t *wfx) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d > delta) return;
    const uint64_t den = (uint64_t)(L - d);
    const uint64_t nhi = (uint64_t)L >> 12, nlo = (uint64_t)L << 52;
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
    wfx[d] = q;
}

// per host thread: accumulators, work counter and weights
struct Star4Ws {
    DevBuf acc, wfx, hist;
};
thread_local Star4Ws t_s4;

std::mutex g_s4_mu;  // builds of the heavy ranks

}  // namespace

// The heavy-leaf ranks of a graph's incidence entries, built on first use
// (one byte per entry, kept with the graph).
tm_status tm_star4_ranks(tm_graph *g, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_s4_mu);
    if (g->s4_rank.p || g->m_nl == 0) return TM_OK;
    const int64_t U = g->U, nr = 2 * U, n = g->n;
    DevBuf keys, vals, cnt, beg, len, rank;
    TM_TRY(keys.alloc((size_t)(nr > 0 ? nr : 1) * 8));
    TM_TRY(vals.alloc((size_t)(nr > 0 ? nr : 1) * 4));
    TM_TRY(cnt.alloc(64));
    TM_TRY(beg.alloc((size_t)n * 8));
    TM_TRY(len.alloc((size_t)n * 8));
    TM_TRY(rank.alloc((size_t)2 * g->m_nl));
    hipLaunchKernelGGL(k_s4_zero, dim3(1), dim3(64), 0, st, cnt.as<uint64_t>(), (int64_t)1);
    hipLaunchKernelGGL(k_s4_zero, dim3(tm_blocks(n, 256)), dim3(256), 0, st, len.as<uint64_t>(), n);
    hipLaunchKernelGGL(k_s4_records, dim3(tm_blocks(g->ph_cap, 256)), dim3(256), 0, st, g->ph_slot.as<PairSlot>(),
                       g->ph_cap, cnt.as<unsigned long long>(), keys.as<uint64_t>(), vals.as<uint32_t>());
    TM_HIP(hipGetLastError());
    TM_TRY(tm_radix_sort(keys.as<uint64_t>(), vals.as<uint32_t>(), nr, 32 + tm_bitlen((uint64_t)n), st));
    hipLaunchKernelGGL(k_s4_segments, dim3(tm_blocks(nr, 256)), dim3(256), 0, st, keys.as<uint64_t>(), nr,
                       beg.as<int64_t>(), len.as<int64_t>());
    hipLaunchKernelGGL(k_s4_lengths, dim3(tm_blocks(n, 256)), dim3(256), 0, st, beg.as<int64_t>(),
                       len.as<int64_t>(), n);
    hipLaunchKernelGGL(k_s4_rank, dim3(tm_blocks(2 * g->m_nl, 256)), dim3(256), 0, st, dev_view(g),
                       vals.as<uint32_t>(), beg.as<int64_t>(), len.as<int64_t>(), rank.as<uint8_t>());
    TM_HIP(hipGetLastError());
    TM_HIP(hipStreamSynchronize(st));
    g->s4_rank.p = rank.p;
    g->s4_rank.bytes = rank.bytes;
    g->s4_rank.cap = rank.cap;
    rank.p = nullptr;
    rank.bytes = rank.cap = 0;
    g->device_bytes += (int64_t)g->s4_rank.bytes;
    return TM_OK;
}

// The center and directions of a motif of this shape, or false.
bool tm_star4_shape(const tm_motif *M, uint32_t d[4]) {
    if (!M || M->l != 4) return false;
    for (int x = 0; x < 2; ++x) {  // the center is node 0 or node 1 (edge 0 is (0, 1))
        int leaf[4];
        bool ok = true;
        for (int k = 0; k < 4 && ok; ++k) {
            const int u = M->src[k], v = M->dst[k];
            if (u == x) {
                d[k] = 0;
                leaf[k] = v;
            } else if (v == x) {
                d[k] = 1;
                leaf[k] = u;
            } else {
                ok = false;
            }
        }
        ok = ok && leaf[0] == leaf[1] && leaf[2] != leaf[0] && leaf[3] != leaf[0] && leaf[2] != leaf[3];
        if (ok) return true;
    }
    return false;
}

// Counts (mode 0), counts and fixed-point weighted sums (mode 1) or counts
// and the duration histogram (mode 2, hist_dev: delta + 1 bins {lo, hi}) of
// a star motif of tm_star4_shape; windowed as Star4Args.  out[4]: count
// lo/hi, weight lo/hi (host).
tm_status tm_star4_run(const tm_graph *g, const tm_motif *M, int mode, int64_t delta, int windowed, int64_t s, int64_t L,
                       uint64_t seed, double p, uint64_t out[4], uint64_t *hist_dev, hipStream_t st) {
    uint32_t d[4];
    if (!tm_star4_shape(M, d)) return TM_EUNSUPPORTED;
    out[0] = out[1] = out[2] = out[3] = 0;
    if (g->m_nl == 0) return TM_OK;
    TM_TRY(tm_star4_ranks(const_cast<tm_graph *>(g), st));
    Star4Ws &W = t_s4;
    TM_TRY(W.acc.reserve(64));
    if (mode == MODE_HIST)
        hipLaunchKernelGGL(k_s4_zero, dim3(tm_blocks(2 * (delta + 1), 256)), dim3(256), 0, st, hist_dev,
                           2 * (delta + 1));
    hipLaunchKernelGGL(k_s4_zero, dim3(1), dim3(64), 0, st, W.acc.as<uint64_t>(), (int64_t)8);
    Star4Args a;
    a.delta = delta;
    a.windowed = windowed;
    a.s = s;
    a.L = L;
    a.seed = seed;
    a.p = p;
    for (int k = 0; k < 4; ++k) a.d[k] = d[k];
    a.wfx = nullptr;
    a.hist = hist_dev;
    a.out = W.acc.as<uint64_t>();
    a.counter = W.acc.as<unsigned long long>() + 4;
    a.rank = g->s4_rank.as<uint8_t>();
    a.n_entries = 2 * g->m_nl;
    if (mode == MODE_WEIGHT) {
        TM_TRY(W.wfx.reserve((size_t)(delta + 1) * 8));
        hipLaunchKernelGGL(k_s4_weights, dim3(tm_blocks(delta + 1, 256)), dim3(256), 0, st, delta, L,
                           W.wfx.as<uint64_t>());
        a.wfx = W.wfx.as<uint64_t>();
    }
    int ncu = 0;
    TM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, g->device));
    if (ncu <= 0) ncu = 256;
    int64_t nb = tm_blocks(a.n_entries, S4_TPB);
    if (nb > (int64_t)ncu * 8) nb = (int64_t)ncu * 8;
    static const char *names[3] = {"star4_count", "star4_weight", "star4_hist"};
    void *tok = tm_prof_begin(names[mode], st);
    if (mode == MODE_COUNT)
        hipLaunchKernelGGL(k_star4<MODE_COUNT>, dim3((unsigned)nb), dim3(S4_TPB), 0, st, dev_view(g), a);
    else if (mode == MODE_WEIGHT)
        hipLaunchKernelGGL(k_star4<MODE_WEIGHT>, dim3((unsigned)nb), dim3(S4_TPB), 0, st, dev_view(g), a);
    else
        hipLaunchKernelGGL(k_star4<MODE_HIST>, dim3((unsigned)nb), dim3(S4_TPB), 0, st, dev_view(g), a);
    TM_HIP(hipGetLastError());
    tm_prof_end(tok, st);
    TM_HIP(hipMemcpyAsync(out, W.acc.p, 32, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    return TM_OK;
}

void tm_star4_release_thread_ws() {
    t_s4.acc.release();
    t_s4.wfx.release();
    t_s4.hist.release();
}

int64_t tm_star4_bytes(const tm_graph *g, int64_t delta) {
    (void)g;
    return 256 + (delta + 1) * 8;  // accumulators and work counter, weights
}

int64_t tm_star4_build_bytes(const tm_graph *g) {
    if (g->s4_rank.p || g->m_nl == 0) return 0;
    const int64_t nr = 2 * g->U;
    // records, their sort, 64 B of counter, node segments, and the ranks
    // themselves (kept with the graph)
    return (nr > 0 ? nr : 1) * 12 + tm_radix_sort_bytes(nr) + 256 + 16 * g->n + 2 * g->m_nl;
}
