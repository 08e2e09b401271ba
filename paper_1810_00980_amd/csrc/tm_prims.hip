// Device primitives: exclusive prefix sum and a stable LSD radix sort.
//
// The radix sort orders (key, value) pairs by 8-bit digits, least
// significant first.  Each pass counts digits per 2048-key tile, turns the
// (digit, tile) count table into output offsets with one prefix sum, and
// scatters every tile stably: the tile is read in 8 rounds of 256 keys; in a
// round, a lane finds the lanes of its wavefront holding the same digit with
// eight 64-lane ballots, ranks itself among them, and the four wavefronts of
// the work-group combine their per-digit counts through LDS.  Stability (equal
// keys keep their input order) is what makes the per-node incidence lists come
// out time-ordered when they are sorted by node after the time sort.
#include "tm_common.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ inline int64_t wave_incl_scan(int64_t x, int lane) {
#pragma unroll
    for (int o = 1; o < TM_WAVE; o <<= 1) {
        int64_t y = __shfl_up(x, o, TM_WAVE);
        if (lane >= o) x += y;
    }
    return x;
}

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ inline int64_t block_excl_scan(int64_t x, int64_t *lds4, int64_t *total) {
    int tid = threadIdx.x, lane = tid & (TM_WAVE - 1), w = tid / TM_WAVE;
    int64_t inc = wave_incl_scan(x, lane);
    if (lane == TM_WAVE - 1) lds4[w] = inc;
    __syncthreads();
    int64_t base = 0, all = 0;
    for (int i = 0; i < SCAN_THREADS / TM_WAVE; ++i) {
        if (i < w) base += lds4[i];
        all += lds4[i];
    }
    __syncthreads();
    *total = all;
    return base + inc - x;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_local(int64_t *d, int64_t n, int64_t *bsum) {
    __shared__ int64_t lds4[SCAN_THREADS / TM_WAVE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + i;
        v[i] = idx < n ? d[idx] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_excl_scan(s, lds4, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + i;
        if (idx < n) d[idx] = ex;
        ex += v[i];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_add(int64_t *d, int64_t n, const int64_t *bsum) {
    int64_t add = bsum[blockIdx.x];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * SCAN_THREADS;
        if (idx < n) d[idx] += add;
    }
}

__global__ void k_copy1(int64_t *dst, const int64_t *src) { dst[0] = src[0]; }

// ----------------------------------------------------------- radix sort

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
constexpr int RS_WAVES = RS_THREADS / TM_WAVE;

__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint64_t *keys, int64_t n, int shift,
                                                       int64_t ntiles, int64_t *counts) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int64_t idx = base + (int64_t)r * RS_THREADS + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint64_t *kin, const uint32_t *vin,
                                                          uint64_t *kout, uint32_t *vout, int64_t n,
                                                          int shift, int64_t ntiles,
                                                          const int64_t *offsets) {
    __shared__ int64_t dbase[256];
    __shared__ uint32_t wcnt[RS_WAVES][256];
    __shared__ uint32_t dtot[256];
    const int tid = threadIdx.x, lane = tid & (TM_WAVE - 1), w = tid / TM_WAVE;
    dbase[tid] = offsets[(int64_t)tid * ntiles + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        for (int i = tid; i < RS_WAVES * 256; i += RS_THREADS) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        int64_t idx = base + (int64_t)r * RS_THREADS + tid;
        bool valid = idx < n;
        uint64_t key = valid ? kin[idx] : 0;
        uint32_t val = valid ? vin[idx] : 0;
        int d = (int)((key >> shift) & 0xFF);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            unsigned long long bm = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bm : ~bm;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t run = 0;
            for (int ww = 0; ww < RS_WAVES; ++ww) {
                uint32_t c = wcnt[ww][tid];
                wcnt[ww][tid] = run;
                run += c;
            }
            dtot[tid] = run;
        }
        __syncthreads();
        if (valid) {
            int64_t p = dbase[d] + wcnt[w][d] + rank;
            kout[p] = key;
            vout[p] = val;
        }
        __syncthreads();
        dbase[tid] += dtot[tid];
        __syncthreads();
    }
}

}  // namespace

namespace {

// Block sums of every level of the scan hierarchy, per host thread, grown on
// demand: a scan then neither allocates nor waits, so a chain of scans and
// kernels on one stream runs without host round trips.  A host thread issues
// its scans on one stream at a time (every library call finishes its work
// before returning), so the next scan's writes come after this one's reads.
thread_local DevBuf t_scan_ws;

int64_t scan_ws_elems(int64_t n) {
    int64_t tot = 0;
    while (true) {
        const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
        tot += nb;
        if (nb <= 1) return tot;
        n = nb;
    }
}

tm_status scan_levels(int64_t *d, int64_t n, int64_t *d_total, int64_t *ws, hipStream_t st) {
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    int64_t *bsum = ws;
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, d, n, bsum);
    TM_HIP(hipGetLastError());
    if (nb > 1) {
        TM_TRY(scan_levels(bsum, nb, d_total, ws + nb, st));
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, d, n, bsum);
        TM_HIP(hipGetLastError());
    } else if (d_total) {
        hipLaunchKernelGGL(k_copy1, dim3(1), dim3(1), 0, st, d_total, bsum);
        TM_HIP(hipGetLastError());
    }
    return TM_OK;
}

}  // namespace

tm_status tm_scan_i64(int64_t *d, int64_t n, int64_t *d_total, hipStream_t st) {
    if (n <= 0) {
        if (d_total) TM_HIP(hipMemsetAsync(d_total, 0, sizeof(int64_t), st));
        return TM_OK;
    }
    const size_t need = (size_t)scan_ws_elems(n) * sizeof(int64_t);
    if (t_scan_ws.bytes < need) {
        // earlier scans of this thread may still read the old buffer
        TM_HIP(hipStreamSynchronize(st));
        TM_TRY(t_scan_ws.reserve(need));
    }
    return scan_levels(d, n, d_total, t_scan_ws.as<int64_t>(), st);
}

tm_status tm_radix_sort(uint64_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t st) {
    if (n <= 1 || bits <= 0) return TM_OK;
    int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    DevBuf k2, v2, cnt;
    TM_TRY(k2.alloc((size_t)n * sizeof(uint64_t)));
    TM_TRY(v2.alloc((size_t)n * sizeof(uint32_t)));
    TM_TRY(cnt.alloc((size_t)ntiles * 256 * sizeof(int64_t)));
    uint64_t *ka = keys, *kb = k2.as<uint64_t>();
    uint32_t *va = vals, *vb = v2.as<uint32_t>();
    int passes = (bits + 7) / 8;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = ps * 8;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, st, ka, n, shift, ntiles,
                           cnt.as<int64_t>());
        TM_HIP(hipGetLastError());
        TM_TRY(tm_scan_i64(cnt.as<int64_t>(), ntiles * 256, nullptr, st));
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, st, ka, va, kb, vb, n,
                           shift, ntiles, cnt.as<int64_t>());
        TM_HIP(hipGetLastError());
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        TM_HIP(hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
        TM_HIP(hipMemcpyAsync(vals, va, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    }
    TM_HIP(hipStreamSynchronize(st));
    return TM_OK;
}

void tm_prims_release_thread_ws() { t_scan_ws.release(); }

int64_t tm_scan_ws_bytes(int64_t n) { return n > 0 ? scan_ws_elems(n) * (int64_t)sizeof(int64_t) : 0; }

int64_t tm_radix_sort_bytes(int64_t n) {
    if (n <= 1) return 0;
    const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    return n * (int64_t)(sizeof(uint64_t) + sizeof(uint32_t)) + ntiles * 256 * (int64_t)sizeof(int64_t) +
           tm_scan_ws_bytes(ntiles * 256);
}
