// Exact-count tables: the exact 2-node and star counts of an anchor as range
// sums over its own pair timeline.
//
// For an anchor entry i of x's combined list (other endpoint y1, direction
// d1, time t1) and its horizon H, the instances whose first edge is i and
// whose other two edges also touch x are, per class (the definitions of a
// motif delta-instance, Sec. 2; middles strictly between in time):
//   2-node (all three on {x, y1}):  last edges j of the pair P = {x, y1} in
//        (t1, H], middles of P in (t1, tj)
//   star B (last edge on P, middle elsewhere) and star A (middle on P, last
//        edge elsewhere)
// and the fourth star class (middle on the last edge's pair) backwards from
// the last edge.  With, for a time t,
//   M_d(t) / M+_d(t)  entries of P of direction d (as seen from x) before t
//                     / up to t,
//   N_d(t) / N+_d(t)  the same over all of x's list,
// every count is a sum over the entries e of P inside a time range of one of
// M_d(t_e), N_d(t_e) or N+_d(t_e) - M+_d(t_e), split by e's own direction,
// minus a product of range sizes and point values.  This file stores, per
// pair entry and for each endpoint's view, global prefix sums of those six
// values split by the entry's direction (12 per view), so that each range
// sum is the difference of two rows.
#include "tm_common.h"

#include <limits.h>

#include "tm_sweep_dev.h"

namespace {

using namespace sweepdev;

constexpr int TPB = 256;

__global__ void k_ex_dir0(const uint32_t *nd, int64_t len, int64_t *f) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < len) f[q] = (nd[q] >> 31) ? 0 : 1;
}

// first position in [lo, hi) with time >= t (lower) or > t (upper)
__device__ inline int64_t list_lower(const int64_t *tv, int64_t lo, int64_t hi, int64_t t) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (tv[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ inline int64_t list_upper(const int64_t *tv, int64_t lo, int64_t hi, int64_t t) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (tv[mid] <= t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The bounds of the tie group of entry q (time t = tv[q]) in a list,
// found by galloping outward from q: one or two loads when t has no ties,
// instead of a binary search over the whole list.
// first index in [lo, q] with tv >= t
__device__ inline int64_t tie_lower(const int64_t *tv, int64_t lo, int64_t q, int64_t t) {
    int64_t hi = q, step = 1, l = lo;  // tv[hi] >= t
    while (true) {
        const int64_t c = hi - step;
        if (c < lo) break;
        if (tv[c] < t) {
            l = c + 1;
            break;
        }
        hi = c;
        step <<= 1;
    }
    return list_lower(tv, l, hi, t);
}

// first index in [q, end) with tv > t (end if none)
__device__ inline int64_t tie_upper(const int64_t *tv, int64_t q, int64_t end, int64_t t) {
    int64_t lo = q, step = 1, h = end;  // tv[lo] <= t
    while (true) {
        const int64_t c = lo + step;
        if (c >= end) break;
        if (tv[c] > t) {
            h = c;
            break;
        }
        lo = c;
        step <<= 1;
    }
    return list_upper(tv, lo + 1, h, t);
}

// values of one pair entry slot in both views, column-major:
// cols[(view * 12 + d_e * 6 + c) * S + slot], c = M_0, M_1, N_0, N_1,
// N+_0 - M+_0, N+_1 - M+_1 (directions as seen from the view's endpoint)
__global__ void k_ex_values(DevGraph G, const uint32_t *ent_nl, const uint32_t *inc_pos, const int64_t *nl_pos,
                            const int64_t *c0x, int64_t S, uint64_t *cols) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    uint64_t v[2][12];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
#pragma unroll
        for (int c = 0; c < 12; ++c) v[w][c] = 0;
    }
    uint32_t nlk = ent_nl[s];
    if (nlk != ~0u) {
        int64_t k = nl_pos[nlk];
        uint32_t src = (uint32_t)G.es_src[k], dst = (uint32_t)G.es_dst[k];
        int64_t t = G.es_t[k];
        uint32_t a = src < dst ? src : dst, b = src < dst ? dst : src;
        PairView pv;
        (void)pair_find(G, a, b, pv);
        // tie group of t in the pair: [gs, ge), with the a -> b counts before
        int64_t ca_gs, ca_ge;
        {
            int64_t c[2];
            pv.lt(G, t, c);
            ca_gs = c[0];
            int64_t gs = c[0] + c[1];
            pv.le(G, t, c);
            ca_ge = c[0];
            int64_t ge = c[0] + c[1];
            const bool ab = src == a;  // the edge runs a -> b
            // view 0 (x = a): direction 0 = a -> b; view 1 (x = b): swapped
            const int64_t M[2][2] = {{ca_gs, gs - ca_gs}, {gs - ca_gs, ca_gs}};
            const int64_t Mp[2][2] = {{ca_ge, ge - ca_ge}, {ge - ca_ge, ca_ge}};
            const uint32_t de[2] = {ab ? 0u : 1u, ab ? 1u : 0u};
            const uint32_t xs[2] = {a, b};
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                // the edge's entry in x's list: side 0 when x is its source
                int64_t q = inc_pos[2 * (int64_t)nlk + ((xs[w] == src) ? 0 : 1)];
                int64_t ls = G.inc_off[xs[w]], lend = G.inc_off[xs[w] + 1];
                int64_t lgs = tie_lower(G.inc_t, ls, q, t);
                int64_t lge = tie_upper(G.inc_t, q, lend, t);
                int64_t n0 = c0x[lgs] - c0x[ls], n1 = (lgs - ls) - n0;
                int64_t n0p = c0x[lge] - c0x[ls], n1p = (lge - ls) - n0p;
                const int64_t val[6] = {M[w][0], M[w][1], n0, n1, n0p - Mp[w][0], n1p - Mp[w][1]};
#pragma unroll
                for (int c = 0; c < 6; ++c) v[w][de[w] * 6 + c] = (uint64_t)val[c];
            }
        }
    }
#pragma unroll
    for (int w = 0; w < 2; ++w) {
#pragma unroll
        for (int c = 0; c < 12; ++c) cols[(int64_t)(w * 12 + c) * S + s] = v[w][c];
    }
}

// column-major prefix sums -> rows[(view * S + slot) * 12 + c].  The columns
// were scanned as one array, so each value less its column's first one is
// the column's own exclusive prefix.
// A block moves EX_T slots of one view through LDS: it reads the 12 column
// runs coalesced and writes the 12 * EX_T row words as one contiguous run.
constexpr int EX_T = 256;
__global__ void __launch_bounds__(EX_T) k_ex_rows(const uint64_t *cols, int64_t S, uint64_t *rows) {
    __shared__ uint64_t tile[EX_T * 13];  // rows padded to 13 words against bank conflicts
    const int w = (int)blockIdx.y;
    const int64_t s0 = (int64_t)blockIdx.x * EX_T;
    const int64_t ns = (S - s0) < EX_T ? (S - s0) : EX_T;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const uint64_t *col = cols + (int64_t)(w * 12 + c) * S;
        if (threadIdx.x < ns) tile[threadIdx.x * 13 + c] = col[s0 + threadIdx.x] - col[0];
    }
    __syncthreads();
    uint64_t *out = rows + ((int64_t)w * S + s0) * 12;
    for (int k = threadIdx.x; k < (int)ns * 12; k += EX_T) out[k] = tile[(k / 12) * 13 + k % 12];
}

}  // namespace

tm_status tm_build_exact_tables(tm_graph *g, const uint32_t *ent_nl, const uint32_t *inc_pos, const int64_t *nl_pos,
                                hipStream_t st) {
    g->has_ex = 0;
    const int64_t len = 2 * g->m_nl;
    const int64_t S = g->m_nl + g->U;
    if (len == 0) return TM_OK;
    // the rows, plus the column-major build copy, within a quarter of free memory
    size_t need = (size_t)S * 2 * 12 * 8 * 2 + (size_t)(len + 1) * 8;
    size_t fr = 0, tot = 0;
    TM_HIP(hipMemGetInfo(&fr, &tot));
    if (need > fr / 4) return TM_OK;
    TM_TRY(g->ex_c0x.alloc((size_t)(len + 1) * 8));
    hipLaunchKernelGGL(k_ex_dir0, dim3(tm_blocks(len, TPB)), dim3(TPB), 0, st, g->inc_nd.as<uint32_t>(), len,
                       g->ex_c0x.as<int64_t>());
    TM_HIP(hipGetLastError());
    TM_TRY(tm_scan_i64(g->ex_c0x.as<int64_t>(), len, g->ex_c0x.as<int64_t>() + len, st));
    DevBuf cols;
    TM_TRY(cols.alloc((size_t)S * 24 * 8));
    hipLaunchKernelGGL(k_ex_values, dim3(tm_blocks(S, TPB)), dim3(TPB), 0, st, dev_view(g), ent_nl, inc_pos, nl_pos,
                       g->ex_c0x.as<int64_t>(), S, cols.as<uint64_t>());
    TM_HIP(hipGetLastError());
    // one exclusive scan over the 24 columns back to back: column c's prefix
    // plus the total of the columns before it, which k_ex_rows subtracts
    TM_TRY(tm_scan_i64(cols.as<int64_t>(), 24 * S, nullptr, st));
    TM_TRY(g->ex_rows.alloc((size_t)S * 24 * 8));
    hipLaunchKernelGGL(k_ex_rows, dim3((unsigned)((S + EX_T - 1) / EX_T), 2), dim3(EX_T), 0, st, cols.as<uint64_t>(), S,
                       g->ex_rows.as<uint64_t>());
    TM_HIP(hipGetLastError());
    TM_HIP(hipStreamSynchronize(st));
    g->ex_S = S;
    g->has_ex = 1;
    return TM_OK;
}
