// Graph ingestion: validation, time normalisation (times start at 0, as
// Algorithm 1 assumes), a stable device radix sort by time, and per-node
// time-sorted incidence lists built by stable sorts on node ids.
#include "tm_common.h"

#include <limits.h>
#include <string.h>

namespace {

constexpr int TPB = 256;

__global__ void k_validate(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t m, int32_t n,
                           int32_t *bad, long long *tmin, long long *tmax) {
    __shared__ long long smin[TPB], smax[TPB];
    long long lo = LLONG_MAX, hi = LLONG_MIN;
    int b = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = src[i], d = dst[i];
        b |= (s < 0) | (s >= n) | (d < 0) | (d >= n);
        long long x = t[i];
        lo = x < lo ? x : lo;
        hi = x > hi ? x : hi;
    }
    if (b) atomicOr(bad, 1);
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = smin[threadIdx.x + s] < smin[threadIdx.x] ? smin[threadIdx.x + s] : smin[threadIdx.x];
            smax[threadIdx.x] = smax[threadIdx.x + s] > smax[threadIdx.x] ? smax[threadIdx.x + s] : smax[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(tmin, smin[0]);
        atomicMax(tmax, smax[0]);
    }
}

__global__ void k_time_keys(const int64_t *t, int64_t m, int64_t tmin, uint64_t *keys, uint32_t *vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) {
        keys[i] = (uint64_t)(t[i] - tmin);
        vals[i] = (uint32_t)i;
    }
}

__global__ void k_gather_sorted(const int32_t *src, const int32_t *dst, const uint64_t *keys, const uint32_t *vals,
                                int64_t m, int32_t *es_src, int32_t *es_dst, int64_t *es_t, int64_t *pos_of,
                                int64_t *nl_flag) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) {
        uint32_t e = vals[k];
        int32_t s = src[e], d = dst[e];
        es_src[k] = s;
        es_dst[k] = d;
        es_t[k] = (int64_t)keys[k];
        pos_of[e] = k;
        nl_flag[k] = (s != d) ? 1 : 0;
    }
}

__global__ void k_compact_nl(const int64_t *flag_scan, const int32_t *es_src, const int32_t *es_dst, int64_t m,
                             int64_t *nl_pos) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m && es_src[k] != es_dst[k]) nl_pos[flag_scan[k]] = k;
}

// keys = node of each non-self-loop edge (src when which == 0, dst when 1)
__global__ void k_node_keys(const int64_t *nl_pos, int64_t m_nl, const int32_t *es_node, uint64_t *keys,
                            uint32_t *vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m_nl) {
        keys[i] = (uint64_t)es_node[nl_pos[i]];
        vals[i] = (uint32_t)i;
    }
}

__global__ void k_fill_list(const uint32_t *vals, int64_t m_nl, const int64_t *nl_pos, const int32_t *es_other,
                            const int64_t *es_t, int32_t *nbr, int64_t *tl) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m_nl) {
        int64_t k = nl_pos[vals[j]];
        nbr[j] = es_other[k];
        tl[j] = es_t[k];
    }
}

// off[v] = first j with keys[j] >= v * scale, v = 0..n
__global__ void k_lower_bound(const uint64_t *keys, int64_t len, int64_t n, uint64_t scale, int64_t *off) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v <= n) {
        uint64_t target = (uint64_t)v * scale;
        int64_t lo = 0, hi = len;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < target) lo = mid + 1;
            else hi = mid;
        }
        off[v] = lo;
    }
}

// distinct directed pairs: each unordered pair adds one per direction that
// has an edge (its sentinel entry holds the a -> b total)
__global__ void k_dir_pairs(const int64_t *ubeg, const PairEnt *ent, int64_t U, unsigned long long *out) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= U) return;
    const int64_t n = ubeg[p + 1] - ubeg[p];
    const int64_t ab = ent[ubeg[p] + p + n].c0;
    atomicAdd(out, (unsigned long long)((ab > 0 ? 1 : 0) + (n - ab > 0 ? 1 : 0)));
}

__global__ void k_set1(int64_t *p, int64_t v) { p[0] = v; }

__global__ void k_inc_keys(const int64_t *nl_pos, int64_t m_nl, const int32_t *es_src, const int32_t *es_dst,
                           uint64_t *keys, uint32_t *vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m_nl) {
        int64_t k = nl_pos[i];
        keys[2 * i] = (uint64_t)es_src[k];
        vals[2 * i] = (uint32_t)(2 * i);
        keys[2 * i + 1] = (uint64_t)es_dst[k];
        vals[2 * i + 1] = (uint32_t)(2 * i + 1);
    }
}

__global__ void k_inc_twin(const uint32_t *vals, int64_t len, uint32_t *posv, uint32_t *twin, int pass) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= len) return;
    uint32_t v = vals[j];
    if (pass == 0) posv[v] = (uint32_t)j;
    else twin[j] = posv[v ^ 1u];
}

__global__ void k_inc_rank(const int64_t *inc_off, const uint32_t *nd, int64_t len, int64_t n, int64_t *hi) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= len) return;
    int64_t lo = 0, up = n;  // owner: largest v with inc_off[v] <= j
    while (up - lo > 1) {
        int64_t mid = (lo + up) >> 1;
        if (inc_off[mid] <= j) lo = mid;
        else up = mid;
    }
    int64_t v = lo, y = nd[j] & 0x7FFFFFFFu;
    int64_t dv = inc_off[v + 1] - inc_off[v], dy = inc_off[y + 1] - inc_off[y];
    hi[j] = (dy > dv || (dy == dv && y > v)) ? 1 : 0;
}

// ranked sublists: entry j goes to pos[j] when it is flagged; node offsets
// are the positions of the nodes' first entries
__global__ void k_hi_fill(const int64_t *flag_pos, const int64_t *flag_orig_hi, const uint32_t *nd, const int64_t *tl,
                          int64_t len, uint32_t *hnd, int64_t *ht) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < len && flag_orig_hi[j]) {
        int64_t q = flag_pos[j];
        hnd[q] = nd[j];
        ht[q] = tl[j];
    }
}

__global__ void k_hi_off(const int64_t *inc_off, const int64_t *flag_pos, int64_t n, int64_t len, int64_t n_hi,
                         int64_t *hoff) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x <= n) {
        int64_t o = inc_off[x];
        hoff[x] = o < len ? flag_pos[o] : n_hi;
    }
}

__global__ void k_inc_fill(const uint32_t *vals, int64_t len, const int64_t *nl_pos, const int32_t *es_src,
                           const int32_t *es_dst, const int64_t *es_t, uint32_t *nd, int64_t *tl) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < len) {
        uint32_t v = vals[j];
        int64_t k = nl_pos[v >> 1];
        uint32_t dir = v & 1u;  // 0: this node is the source, 1: the destination
        uint32_t other = dir ? (uint32_t)es_src[k] : (uint32_t)es_dst[k];
        nd[j] = other | (dir << 31);
        tl[j] = es_t[k];
    }
}


__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_slot_init(PairSlot *slots, int64_t cap) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cap) {
        PairSlot z;
        z.key = ~0ull;
        z.t0 = z.base = z.boff = 0;
        z.id = -1;
        z.shift = z.nb = 0;
        z.n = 0;
        slots[i] = z;
    }
}

// unordered pair key (min * n + max) of every non-self-loop edge, in time order
__global__ void k_upair_keys(const int64_t *nl_pos, int64_t m_nl, const int32_t *es_src, const int32_t *es_dst,
                             int64_t n, uint64_t *keys, uint32_t *vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m_nl) {
        int64_t k = nl_pos[i];
        uint64_t u = (uint64_t)es_src[k], v = (uint64_t)es_dst[k];
        keys[i] = (u < v ? u : v) * (uint64_t)n + (u < v ? v : u);
        vals[i] = (uint32_t)i;
    }
}

__device__ inline bool upair_start(const uint64_t *keys, int64_t j) { return j == 0 || keys[j] != keys[j - 1]; }

// after the stable sort by key: pair-start flags and min -> max flags
__global__ void k_upair_flags(const uint64_t *keys, const uint32_t *vals, int64_t m_nl, const int64_t *nl_pos,
                              const int32_t *es_src, const int32_t *es_dst, int64_t *bflag, int64_t *c0) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m_nl) {
        int64_t k = nl_pos[vals[j]];
        bflag[j] = upair_start(keys, j) ? 1 : 0;
        c0[j] = es_src[k] < es_dst[k] ? 1 : 0;
    }
}

__global__ void k_upair_index(const uint64_t *keys, const int64_t *bscan, int64_t m_nl, uint64_t *u_key,
                              int64_t *up_beg) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m_nl && upair_start(keys, j)) {
        int64_t p = bscan[j];
        u_key[p] = keys[j];
        up_beg[p] = j;
    }
}

// entry j of pair p goes to j + p (each earlier pair has one sentinel); the
// last entry of a pair also writes the sentinel after it
__global__ void k_upair_place(const uint64_t *keys, const uint32_t *vals, int64_t m_nl, const int64_t *nl_pos,
                              const int32_t *es_src, const int32_t *es_dst, const int64_t *es_t,
                              const int64_t *bscan, const int64_t *g0, const int64_t *up_beg, PairEnt *ent,
                              uint32_t *ent_nl) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m_nl) return;
    int64_t pid = bscan[j] + (upair_start(keys, j) ? 1 : 0) - 1;
    int64_t b = up_beg[pid];
    int64_t k = nl_pos[vals[j]];
    PairEnt e;
    e.t = es_t[k];
    e.c0 = g0[j] - g0[b];
    ent[j + pid] = e;
    ent_nl[j + pid] = vals[j];
    if (j + 1 == m_nl || keys[j + 1] != keys[j]) {
        PairEnt z;
        z.t = LLONG_MAX;
        z.c0 = e.c0 + (es_src[k] < es_dst[k] ? 1 : 0);
        ent[j + pid + 1] = z;
        ent_nl[j + pid + 1] = ~0u;
    }
}

// copy each pair's metadata and size into its hash slot
__global__ void k_slot_meta(PairSlot *slots, int64_t cap, const PairMeta *pm, const PairBucket *bk) {
    int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= cap) return;
    int32_t id = slots[h].id;
    if (id < 0) return;
    const PairMeta m = pm[id];
    slots[h].t0 = m.t0;
    slots[h].base = m.base;
    slots[h].boff = m.boff;
    slots[h].shift = m.shift;
    slots[h].nb = m.nb;
    slots[h].n = bk[m.boff + m.nb].idx;
}

__global__ void k_pair_hash_insert(const uint64_t *u_key, int64_t U, int64_t n, PairSlot *slots, int64_t cap) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= U) return;
    uint64_t a = u_key[p] / (uint64_t)n, b = u_key[p] % (uint64_t)n;
    uint64_t key = (a << 32) | b;
    uint64_t h = tm_pair_hash(key, cap);
    for (int64_t probe = 0; probe < cap; ++probe) {
        unsigned long long prev = atomicCAS((unsigned long long *)&slots[h].key, ~0ull, (unsigned long long)key);
        if (prev == ~0ull) {
            slots[h].id = (int32_t)p;
            return;
        }
        h = (h + 1) & (uint64_t)(cap - 1);
    }
}

__global__ void k_pair_meta_pack(const int64_t *up_beg, const int64_t *tfirst, const int32_t *meta,
                                 const int64_t *boff, int64_t U, PairMeta *pm) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= U) return;
    PairMeta m;
    m.t0 = tfirst[p];
    m.base = up_beg[p] + p;
    m.boff = boff[p];
    m.shift = meta[2 * p];
    m.nb = meta[2 * p + 1];
    pm[p] = m;
}

// per pair: first time, bucket shift (at most TM_PAIR_BUCKET_DENSITY buckets per entry), count
__global__ void k_pair_bucket_meta(const int64_t *up_beg, const PairEnt *ent, int64_t U, int64_t *tfirst,
                                   int32_t *meta, int64_t *nbk) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= U) return;
    int64_t b = up_beg[p], e = up_beg[p + 1], k = e - b, base = b + p;
    int64_t t0 = ent[base].t, span = ent[base + k - 1].t - t0;
    int64_t target = k * TM_PAIR_BUCKET_DENSITY;  // buckets wanted (nb stays below 2^31)
    if (target > ((int64_t)1 << 30)) target = (int64_t)1 << 30;
    int shift = 0;
    while (shift < 62 && (span >> shift) + 1 > target) ++shift;
    int64_t nb = (span >> shift) + 1;
    tfirst[p] = t0;
    meta[2 * p] = shift;
    meta[2 * p + 1] = (int32_t)nb;
    nbk[p] = nb + 1;  // with sentinel
}

// entry r of pair p is the first entry of buckets (bucket(r-1), bucket(r)]
__global__ void k_pair_bucket_fill(const uint64_t *keys, const int64_t *bscan, const int64_t *up_beg,
                                   const PairEnt *ent, int64_t m_nl, const int64_t *tfirst, const int32_t *meta,
                                   const int64_t *boff, PairBucket *bk) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m_nl) return;
    int64_t p = bscan[j] + (upair_start(keys, j) ? 1 : 0) - 1;
    int64_t b0 = up_beg[p], k = up_beg[p + 1] - b0, r = j - b0, base = b0 + p;
    int shift = meta[2 * p];
    int32_t nb = meta[2 * p + 1];
    int64_t bi = (ent[base + r].t - tfirst[p]) >> shift;
    int64_t bprev = r == 0 ? -1 : ((ent[base + r - 1].t - tfirst[p]) >> shift);
    PairBucket v;
    v.idx = (uint32_t)r;
    v.c0 = (uint32_t)ent[base + r].c0;
    for (int64_t bb = bprev + 1; bb <= bi; ++bb) bk[boff[p] + bb] = v;
    if (r == k - 1) {  // sentinel (bi == nb - 1 here)
        v.idx = (uint32_t)k;
        v.c0 = (uint32_t)ent[base + k].c0;
        bk[boff[p] + nb] = v;
    }
}

tm_status build_node_lists(tm_graph *g, const int64_t *nl_pos, bool by_src, DevBuf &off, DevBuf &nbr, DevBuf &tl,
                           hipStream_t st) {
    int64_t mn = g->m_nl, n = g->n;
    DevBuf keys, vals;
    TM_TRY(keys.alloc((size_t)mn * 8));
    TM_TRY(vals.alloc((size_t)mn * 4));
    TM_TRY(off.alloc((size_t)(n + 1) * 8));
    TM_TRY(nbr.alloc((size_t)mn * 4));
    TM_TRY(tl.alloc((size_t)mn * 8));
    const int32_t *node = by_src ? g->es_src.as<int32_t>() : g->es_dst.as<int32_t>();
    const int32_t *other = by_src ? g->es_dst.as<int32_t>() : g->es_src.as<int32_t>();
    if (mn > 0) {
        hipLaunchKernelGGL(k_node_keys, dim3(tm_blocks(mn, TPB)), dim3(TPB), 0, st, nl_pos, mn, node,
                           keys.as<uint64_t>(), vals.as<uint32_t>());
        TM_HIP(hipGetLastError());
        TM_TRY(tm_radix_sort(keys.as<uint64_t>(), vals.as<uint32_t>(), mn, tm_bitlen((uint64_t)(n - 1)), st));
        hipLaunchKernelGGL(k_fill_list, dim3(tm_blocks(mn, TPB)), dim3(TPB), 0, st, vals.as<uint32_t>(), mn, nl_pos,
                           other, g->es_t.as<int64_t>(), nbr.as<int32_t>(), tl.as<int64_t>());
        TM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_lower_bound, dim3(tm_blocks(n + 1, TPB)), dim3(TPB), 0, st, keys.as<uint64_t>(), mn, n,
                       (uint64_t)1, off.as<int64_t>());
    TM_HIP(hipGetLastError());
    TM_HIP(hipStreamSynchronize(st));
    return TM_OK;
}

tm_status load_impl(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t m, int32_t n_nodes,
                    int32_t on_device, hipStream_t st, tm_graph *g) {
    TM_HIP(hipGetDevice(&g->device));
    g->m = m;
    g->n = n_nodes;
    DevBuf hsrc, hdst, ht;
    DevBuf ent_nl, inc_pos;  // kept for the exact-count tables
    const int32_t *d_src = src, *d_dst = dst;
    const int64_t *d_t = t;
    if (!on_device && m > 0) {
        TM_TRY(hsrc.alloc((size_t)m * 4));
        TM_TRY(hdst.alloc((size_t)m * 4));
        TM_TRY(ht.alloc((size_t)m * 8));
        TM_HIP(hipMemcpyAsync(hsrc.p, src, (size_t)m * 4, hipMemcpyHostToDevice, st));
        TM_HIP(hipMemcpyAsync(hdst.p, dst, (size_t)m * 4, hipMemcpyHostToDevice, st));
        TM_HIP(hipMemcpyAsync(ht.p, t, (size_t)m * 8, hipMemcpyHostToDevice, st));
        d_src = hsrc.as<int32_t>();
        d_dst = hdst.as<int32_t>();
        d_t = ht.as<int64_t>();
    }
    // validation and time range
    DevBuf red;
    TM_TRY(red.alloc(64));
    struct { int32_t bad; int32_t pad; long long tmin, tmax; } h0 = {0, 0, LLONG_MAX, LLONG_MIN}, h1;
    TM_HIP(hipMemcpyAsync(red.p, &h0, sizeof h0, hipMemcpyHostToDevice, st));
    if (m > 0) {
        unsigned nb = tm_blocks(m, TPB);
        if (nb > 4096) nb = 4096;
        char *rb = red.as<char>();
        hipLaunchKernelGGL(k_validate, dim3(nb), dim3(TPB), 0, st, d_src, d_dst, d_t, m, n_nodes, (int32_t *)rb,
                           (long long *)(rb + 8), (long long *)(rb + 16));
        TM_HIP(hipGetLastError());
    }
    TM_HIP(hipMemcpyAsync(&h1, red.p, sizeof h1, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    if (h1.bad) return TM_EINVAL;
    if (m > 0) {
        // t - t_min must not overflow int64
        if (h1.tmin < 0 && h1.tmax > LLONG_MAX + h1.tmin) return TM_EINVAL;
        g->t_min = h1.tmin;
        g->t_span = h1.tmax - h1.tmin;
    }

    // sorted edge array
    TM_TRY(g->es_src.alloc((size_t)m * 4));
    TM_TRY(g->es_dst.alloc((size_t)m * 4));
    TM_TRY(g->es_t.alloc((size_t)m * 8));
    TM_TRY(g->pos_of.alloc((size_t)m * 8));
    DevBuf keys, vals, flag, nl;
    TM_TRY(keys.alloc((size_t)m * 8));
    TM_TRY(vals.alloc((size_t)m * 4));
    TM_TRY(flag.alloc((size_t)(m + 1) * 8));
    if (m > 0) {
        hipLaunchKernelGGL(k_time_keys, dim3(tm_blocks(m, TPB)), dim3(TPB), 0, st, d_t, m, g->t_min,
                           keys.as<uint64_t>(), vals.as<uint32_t>());
        TM_HIP(hipGetLastError());
        TM_TRY(tm_radix_sort(keys.as<uint64_t>(), vals.as<uint32_t>(), m, tm_bitlen((uint64_t)g->t_span), st));
        hipLaunchKernelGGL(k_gather_sorted, dim3(tm_blocks(m, TPB)), dim3(TPB), 0, st, d_src, d_dst,
                           keys.as<uint64_t>(), vals.as<uint32_t>(), m, g->es_src.as<int32_t>(),
                           g->es_dst.as<int32_t>(), g->es_t.as<int64_t>(), g->pos_of.as<int64_t>(),
                           flag.as<int64_t>());
        TM_HIP(hipGetLastError());
    }
    // non-self-loop positions
    DevBuf cnt;  // device scalars read back: [0] a scan total, [1] the directed pair count
    TM_TRY(cnt.alloc(16));
    TM_TRY(tm_scan_i64(flag.as<int64_t>(), m, cnt.as<int64_t>(), st));
    int64_t m_nl = 0;
    TM_HIP(hipMemcpyAsync(&m_nl, cnt.p, 8, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    g->m_nl = m_nl;
    TM_TRY(nl.alloc((size_t)m_nl * 8));
    if (m > 0) {
        hipLaunchKernelGGL(k_compact_nl, dim3(tm_blocks(m, TPB)), dim3(TPB), 0, st, flag.as<int64_t>(),
                           g->es_src.as<int32_t>(), g->es_dst.as<int32_t>(), m, nl.as<int64_t>());
        TM_HIP(hipGetLastError());
    }
    keys.release();
    vals.release();
    hsrc.release();
    hdst.release();
    ht.release();

    // out- and in-lists
    TM_TRY(build_node_lists(g, nl.as<int64_t>(), true, g->out_off, g->out_nbr, g->out_t, st));
    TM_TRY(build_node_lists(g, nl.as<int64_t>(), false, g->in_off, g->in_nbr, g->in_t, st));

    // unordered pair timelines, pair hash and per-pair time buckets
    {
        int64_t n = g->n;
        DevBuf uk, uv, bscan, g0, ukey, ubeg;
        TM_TRY(uk.alloc((size_t)m_nl * 8));
        TM_TRY(uv.alloc((size_t)m_nl * 4));
        TM_TRY(bscan.alloc((size_t)(m_nl + 1) * 8));
        TM_TRY(g0.alloc((size_t)(m_nl + 1) * 8));
        int64_t U = 0;
        if (m_nl > 0) {
            hipLaunchKernelGGL(k_upair_keys, dim3(tm_blocks(m_nl, TPB)), dim3(TPB), 0, st, nl.as<int64_t>(), m_nl,
                               g->es_src.as<int32_t>(), g->es_dst.as<int32_t>(), n, uk.as<uint64_t>(),
                               uv.as<uint32_t>());
            TM_HIP(hipGetLastError());
            TM_TRY(tm_radix_sort(uk.as<uint64_t>(), uv.as<uint32_t>(), m_nl,
                                 tm_bitlen((uint64_t)n * (uint64_t)n - 1), st));
            hipLaunchKernelGGL(k_upair_flags, dim3(tm_blocks(m_nl, TPB)), dim3(TPB), 0, st, uk.as<uint64_t>(),
                               uv.as<uint32_t>(), m_nl, nl.as<int64_t>(), g->es_src.as<int32_t>(),
                               g->es_dst.as<int32_t>(), bscan.as<int64_t>(), g0.as<int64_t>());
            TM_HIP(hipGetLastError());
            TM_TRY(tm_scan_i64(g0.as<int64_t>(), m_nl, nullptr, st));
            TM_TRY(tm_scan_i64(bscan.as<int64_t>(), m_nl, cnt.as<int64_t>(), st));
            TM_HIP(hipMemcpyAsync(&U, cnt.p, 8, hipMemcpyDeviceToHost, st));
            TM_HIP(hipStreamSynchronize(st));
        }
        g->U = U;
        TM_TRY(ukey.alloc((size_t)(U > 0 ? U : 1) * 8));
        TM_TRY(ubeg.alloc((size_t)(U + 1) * 8));
        TM_TRY(g->up_ent.alloc((size_t)(m_nl + U > 0 ? m_nl + U : 1) * sizeof(PairEnt)));
        TM_TRY(ent_nl.alloc((size_t)(m_nl + U > 0 ? m_nl + U : 1) * 4));
        if (m_nl > 0) {
            hipLaunchKernelGGL(k_upair_index, dim3(tm_blocks(m_nl, TPB)), dim3(TPB), 0, st, uk.as<uint64_t>(),
                               bscan.as<int64_t>(), m_nl, ukey.as<uint64_t>(), ubeg.as<int64_t>());
            TM_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_set1, dim3(1), dim3(1), 0, st, ubeg.as<int64_t>() + U, m_nl);
        TM_HIP(hipGetLastError());
        if (m_nl > 0) {
            hipLaunchKernelGGL(k_upair_place, dim3(tm_blocks(m_nl, TPB)), dim3(TPB), 0, st, uk.as<uint64_t>(),
                               uv.as<uint32_t>(), m_nl, nl.as<int64_t>(), g->es_src.as<int32_t>(),
                               g->es_dst.as<int32_t>(), g->es_t.as<int64_t>(), bscan.as<int64_t>(),
                               g0.as<int64_t>(), ubeg.as<int64_t>(), g->up_ent.as<PairEnt>(),
                               ent_nl.as<uint32_t>());
            TM_HIP(hipGetLastError());
        }

        int64_t cap = 1024;
        while (cap < 2 * U) cap <<= 1;
        g->ph_cap = cap;
        TM_TRY(g->ph_slot.alloc((size_t)cap * sizeof(PairSlot)));
        hipLaunchKernelGGL(k_slot_init, dim3(tm_blocks(cap, TPB)), dim3(TPB), 0, st, g->ph_slot.as<PairSlot>(), cap);
        TM_HIP(hipGetLastError());
        DevBuf tfirst, meta, boff;
        TM_TRY(tfirst.alloc((size_t)(U > 0 ? U : 1) * 8));
        TM_TRY(meta.alloc((size_t)(U > 0 ? U : 1) * 8));
        TM_TRY(boff.alloc((size_t)(U + 1) * 8));
        TM_TRY(g->pmeta.alloc((size_t)(U > 0 ? U : 1) * sizeof(PairMeta)));
        int64_t nbk_total = 0;
        if (U > 0) {
            hipLaunchKernelGGL(k_pair_hash_insert, dim3(tm_blocks(U, TPB)), dim3(TPB), 0, st, ukey.as<uint64_t>(), U,
                               n, g->ph_slot.as<PairSlot>(), cap);
            TM_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_pair_bucket_meta, dim3(tm_blocks(U, TPB)), dim3(TPB), 0, st, ubeg.as<int64_t>(),
                               g->up_ent.as<PairEnt>(), U, tfirst.as<int64_t>(), meta.as<int32_t>(),
                               boff.as<int64_t>());
            TM_HIP(hipGetLastError());
            TM_TRY(tm_scan_i64(boff.as<int64_t>(), U, cnt.as<int64_t>(), st));
            TM_HIP(hipMemsetAsync(cnt.as<int64_t>() + 1, 0, 8, st));
            hipLaunchKernelGGL(k_dir_pairs, dim3(tm_blocks(U, TPB)), dim3(TPB), 0, st, ubeg.as<int64_t>(),
                               g->up_ent.as<PairEnt>(), U, (unsigned long long *)(cnt.as<int64_t>() + 1));
            TM_HIP(hipGetLastError());
            int64_t two[2] = {0, 0};
            TM_HIP(hipMemcpyAsync(two, cnt.p, 16, hipMemcpyDeviceToHost, st));
            TM_HIP(hipStreamSynchronize(st));
            nbk_total = two[0];
            g->S = two[1];
        }
        TM_TRY(g->pbk.alloc((size_t)(nbk_total > 0 ? nbk_total : 1) * sizeof(PairBucket)));
        if (U > 0) {
            hipLaunchKernelGGL(k_pair_bucket_fill, dim3(tm_blocks(m_nl, TPB)), dim3(TPB), 0, st, uk.as<uint64_t>(),
                               bscan.as<int64_t>(), ubeg.as<int64_t>(), g->up_ent.as<PairEnt>(), m_nl,
                               tfirst.as<int64_t>(), meta.as<int32_t>(), boff.as<int64_t>(), g->pbk.as<PairBucket>());
            TM_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_pair_meta_pack, dim3(tm_blocks(U, TPB)), dim3(TPB), 0, st, ubeg.as<int64_t>(),
                               tfirst.as<int64_t>(), meta.as<int32_t>(), boff.as<int64_t>(), U,
                               g->pmeta.as<PairMeta>());
            TM_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_slot_meta, dim3(tm_blocks(cap, TPB)), dim3(TPB), 0, st, g->ph_slot.as<PairSlot>(),
                               cap, g->pmeta.as<PairMeta>(), g->pbk.as<PairBucket>());
            TM_HIP(hipGetLastError());
        }
        TM_HIP(hipStreamSynchronize(st));
    }

    // combined incidence lists
    {
        int64_t len = 2 * m_nl, n = g->n;
        DevBuf ik, iv;
        TM_TRY(ik.alloc((size_t)len * 8));
        TM_TRY(iv.alloc((size_t)len * 4));
        TM_TRY(g->inc_nd.alloc((size_t)len * 4));
        TM_TRY(g->inc_t.alloc((size_t)len * 8));
        TM_TRY(g->inc_twin.alloc((size_t)len * 4));
        TM_TRY(g->inc_off.alloc((size_t)(n + 1) * 8));
        if (m_nl > 0) {
            hipLaunchKernelGGL(k_inc_keys, dim3(tm_blocks(m_nl, TPB)), dim3(TPB), 0, st, nl.as<int64_t>(), m_nl,
                               g->es_src.as<int32_t>(), g->es_dst.as<int32_t>(), ik.as<uint64_t>(), iv.as<uint32_t>());
            TM_HIP(hipGetLastError());
            TM_TRY(tm_radix_sort(ik.as<uint64_t>(), iv.as<uint32_t>(), len, tm_bitlen((uint64_t)(n - 1)), st));
            hipLaunchKernelGGL(k_inc_fill, dim3(tm_blocks(len, TPB)), dim3(TPB), 0, st, iv.as<uint32_t>(), len,
                               nl.as<int64_t>(), g->es_src.as<int32_t>(), g->es_dst.as<int32_t>(),
                               g->es_t.as<int64_t>(), g->inc_nd.as<uint32_t>(), g->inc_t.as<int64_t>());
            TM_HIP(hipGetLastError());
            TM_TRY(inc_pos.alloc((size_t)len * 4));
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(k_inc_twin, dim3(tm_blocks(len, TPB)), dim3(TPB), 0, st, iv.as<uint32_t>(), len,
                                   inc_pos.as<uint32_t>(), g->inc_twin.as<uint32_t>(), pass);
                TM_HIP(hipGetLastError());
            }
            TM_HIP(hipStreamSynchronize(st));
        }
        hipLaunchKernelGGL(k_lower_bound, dim3(tm_blocks(n + 1, TPB)), dim3(TPB), 0, st, ik.as<uint64_t>(), len, n,
                           (uint64_t)1, g->inc_off.as<int64_t>());
        TM_HIP(hipGetLastError());
        // ranked sublists
        DevBuf hflag, hpos;
        TM_TRY(hflag.alloc((size_t)(len + 1) * 8));
        TM_TRY(hpos.alloc((size_t)(len + 1) * 8));
        int64_t n_hi = 0;
        if (m_nl > 0) {
            hipLaunchKernelGGL(k_inc_rank, dim3(tm_blocks(len, TPB)), dim3(TPB), 0, st, g->inc_off.as<int64_t>(),
                               g->inc_nd.as<uint32_t>(), len, n, hflag.as<int64_t>());
            TM_HIP(hipGetLastError());
            TM_HIP(hipMemcpyAsync(hpos.p, hflag.p, (size_t)len * 8, hipMemcpyDeviceToDevice, st));
            TM_TRY(tm_scan_i64(hpos.as<int64_t>(), len, cnt.as<int64_t>(), st));
            TM_HIP(hipMemcpyAsync(&n_hi, cnt.p, 8, hipMemcpyDeviceToHost, st));
            TM_HIP(hipStreamSynchronize(st));
        }
        g->n_hi = n_hi;
        TM_TRY(g->hi_nd.alloc((size_t)(n_hi > 0 ? n_hi : 1) * 4));
        TM_TRY(g->hi_t.alloc((size_t)(n_hi > 0 ? n_hi : 1) * 8));
        TM_TRY(g->hi_off.alloc((size_t)(n + 1) * 8));
        if (m_nl > 0) {
            hipLaunchKernelGGL(k_hi_fill, dim3(tm_blocks(len, TPB)), dim3(TPB), 0, st, hpos.as<int64_t>(),
                               hflag.as<int64_t>(), g->inc_nd.as<uint32_t>(), g->inc_t.as<int64_t>(), len,
                               g->hi_nd.as<uint32_t>(), g->hi_t.as<int64_t>());
            TM_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_hi_off, dim3(tm_blocks(n + 1, TPB)), dim3(TPB), 0, st, g->inc_off.as<int64_t>(),
                           hpos.as<int64_t>(), n, len, n_hi, g->hi_off.as<int64_t>());
        TM_HIP(hipGetLastError());
        TM_HIP(hipStreamSynchronize(st));
    }
    if (m_nl > 0 && g->want_ex)
        TM_TRY(tm_build_exact_tables(g, ent_nl.as<uint32_t>(), inc_pos.as<uint32_t>(), nl.as<int64_t>(), st));
    ent_nl.release();
    inc_pos.release();
    const DevBuf *all[] = {&g->es_src, &g->es_dst, &g->es_t, &g->pos_of, &g->out_off, &g->out_nbr, &g->out_t,
                           &g->in_off, &g->in_nbr, &g->in_t,
                           &g->inc_off, &g->inc_nd, &g->inc_t, &g->inc_twin, &g->hi_off, &g->hi_nd, &g->hi_t, &g->up_ent, &g->ph_slot, &g->pmeta, &g->pbk, &g->ex_c0x, &g->ex_rows};
    int64_t tot = 0;
    for (const DevBuf *b : all) tot += (int64_t)b->bytes;
    g->device_bytes = tot;
    return TM_OK;
}

}  // namespace

DevGraph dev_view(const tm_graph *g) {
    DevGraph v;
    v.m = g->m; v.n = g->n; v.m_nl = g->m_nl; v.S = g->S;
    v.es_src = g->es_src.as<int32_t>(); v.es_dst = g->es_dst.as<int32_t>(); v.es_t = g->es_t.as<int64_t>();
    v.out_off = g->out_off.as<int64_t>(); v.out_nbr = g->out_nbr.as<int32_t>(); v.out_t = g->out_t.as<int64_t>();
    v.in_off = g->in_off.as<int64_t>(); v.in_nbr = g->in_nbr.as<int32_t>(); v.in_t = g->in_t.as<int64_t>();
    v.inc_off = g->inc_off.as<int64_t>(); v.inc_nd = g->inc_nd.as<uint32_t>(); v.inc_t = g->inc_t.as<int64_t>();
    v.inc_twin = g->inc_twin.as<uint32_t>();
    v.n_hi = g->n_hi;
    v.hi_off = g->hi_off.as<int64_t>();
    v.hi_nd = g->hi_nd.as<uint32_t>();
    v.hi_t = g->hi_t.as<int64_t>();
    v.ph_slot = g->ph_slot.as<PairSlot>(); v.ph_cap = g->ph_cap;
    v.pmeta = g->pmeta.as<PairMeta>();
    v.pbk = g->pbk.as<PairBucket>();
    v.up_ent = g->up_ent.as<PairEnt>();
    v.has_ex = g->has_ex;
    v.ex_S = g->ex_S;
    v.ex_c0x = g->ex_c0x.as<int64_t>();
    v.ex_rows = g->ex_rows.as<uint64_t>();
    return v;
}

extern "C" tm_status tm_load_graph_ex(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t m,
                                      int32_t n_nodes, uint32_t flags, void *hip_stream, tm_graph **out) {
    if (!out || m < 0 || n_nodes <= 0 || (m > 0 && (!src || !dst || !t))) return TM_EINVAL;
    if (flags & ~(uint32_t)(TM_LOAD_ON_DEVICE | TM_LOAD_NO_EXACT_TABLES)) return TM_EINVAL;
    if (m > (int64_t)INT32_MAX) return TM_EINVAL;  // 32-bit edge indices in the sorts
    LoadCacheScope cache;  // the load's temporaries are kept for the next load on this thread
    tm_graph *g = new (std::nothrow) tm_graph();
    if (!g) return TM_ENOMEM;
    g->want_ex = (flags & TM_LOAD_NO_EXACT_TABLES) ? 0 : 1;
    tm_status s = load_impl(src, dst, t, m, n_nodes, (flags & TM_LOAD_ON_DEVICE) ? 1 : 0, (hipStream_t)hip_stream, g);
    if (s != TM_OK) {
        (void)hipStreamSynchronize((hipStream_t)hip_stream);
        delete g;
        (void)hipGetLastError();
        return s;
    }
    *out = g;
    return TM_OK;
}

extern "C" tm_status tm_load_graph(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t m,
                                   int32_t n_nodes, int32_t on_device, void *hip_stream, tm_graph **out) {
    return tm_load_graph_ex(src, dst, t, m, n_nodes, on_device ? (uint32_t)TM_LOAD_ON_DEVICE : 0u, hip_stream, out);
}

extern "C" void tm_free_graph(tm_graph *g) {
    if (!g) return;
    {
        std::shared_lock<std::shared_mutex> lk(tm_capture_lock());
        (void)hipDeviceSynchronize();
    }
    tm_batch_forget(g);
    delete g;
}

extern "C" tm_status tm_graph_info_get(const tm_graph *g, tm_graph_info *info) {
    if (!g || !info) return TM_EINVAL;
    info->m = g->m;
    info->n = g->n;
    info->t_min = g->t_min;
    info->t_span = g->t_span;
    info->n_pairs = g->S;
    info->device_bytes = g->device_bytes;
    info->exact_table_bytes = (int64_t)(g->ex_c0x.bytes + g->ex_rows.bytes);
    return TM_OK;
}
