// C-ABI entry points for counting and estimation, the window partitioner
// and the per-window Bernoulli sampler (Algorithm 1, Sec. 4).
#include "tm_common.h"

#include <limits.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

// ---------------------------------------------------------------- profiling
namespace {
struct ProfEvent {
    const char *name;
    hipEvent_t a, b;
    uint64_t pass;
};
struct ProfState {
    std::mutex mu;
    bool on = false;
    bool serial = false;
    std::vector<ProfEvent> pending;
    std::map<std::string, std::pair<double, int64_t>> total;
    uint64_t next_pass = 0;
};
ProfState &prof() {
    static ProfState s;
    return s;
}
}  // namespace

bool tm_prof_serial() {
    ProfState &P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    return P.on && P.serial;
}

uint64_t tm_prof_pass() {
    ProfState &P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    return ++P.next_pass;
}

void *tm_prof_begin(const char *name, hipStream_t st, uint64_t pass) {
    ProfState &P = prof();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        if (!P.on) return nullptr;
    }
    ProfEvent *e = new (std::nothrow) ProfEvent{name, nullptr, nullptr, pass};
    if (!e) return nullptr;
    if (tm_locked_call([&] { return hipEventCreate(&e->a); }) != hipSuccess ||
        tm_locked_call([&] { return hipEventCreate(&e->b); }) != hipSuccess || hipEventRecord(e->a, st) != hipSuccess) {
        (void)hipGetLastError();
        delete e;
        return nullptr;
    }
    return e;
}

void tm_prof_end(void *token, hipStream_t st) {
    if (!token) return;
    ProfEvent *e = static_cast<ProfEvent *>(token);
    if (hipEventRecord(e->b, st) != hipSuccess) {
        (void)hipGetLastError();
        delete e;
        return;
    }
    ProfState &P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.pending.push_back(*e);
    delete e;
}

void tm_prof_collect() {
    ProfState &P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    // longest kernel of each pass
    std::map<uint64_t, std::pair<double, const char *>> crit;
    for (ProfEvent &e : P.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
            auto &t = P.total[e.name];
            t.first += ms;
            t.second += 1;
            if (e.pass) {
                auto &c = crit[e.pass];
                if (!c.second || ms > c.first) c = {ms, e.name};
            }
        }
        (void)hipGetLastError();
        (void)tm_locked_call([&] { return hipEventDestroy(e.a); });
        (void)tm_locked_call([&] { return hipEventDestroy(e.b); });
    }
    P.pending.clear();
    for (auto &kv : crit) {
        auto &t = P.total[std::string("crit:") + kv.second.second];
        t.first += kv.second.first;
        t.second += 1;
    }
}

tm_status tm_sweep_census_impl(const tm_graph *g, int64_t delta, int64_t s, int64_t L, double p, uint64_t seed,
                               tm_census *c, hipStream_t st);

namespace {

constexpr int TPB = 256;

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// multiplications by fixed odd constants, a mix of the high halves with the
// other two counter words and the key, and a word permutation; the two key
// words advance by the golden-ratio and sqrt(3)-1 Weyl increments after every
// round but the last.
__host__ __device__ inline void philox10(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3, uint32_t k0,
                                         uint32_t k1) {
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

// 64-bit draw for (seed, index j, estimator k, domain): counter words
// (j low, j high, k, domain), key words (seed low, seed high); the draw is
// word1 * 2^32 + word0.
__host__ __device__ inline uint64_t tm_draw(uint64_t seed, uint64_t j, uint32_t k, uint32_t domain) {
    uint32_t x0 = (uint32_t)j, x1 = (uint32_t)(j >> 32), x2 = k, x3 = domain;
    philox10(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
    return ((uint64_t)x1 << 32) | (uint64_t)x0;
}

// keep window j of estimator (seed) when (draw >> 11) * 2^-53 < p
__device__ inline bool tm_keep(uint64_t seed, uint64_t j, double p) {
    uint64_t x = tm_draw(seed, j, 0, 1);
    double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);
    return u < p;
}

__global__ void k_shift(uint64_t seed, int64_t L, int64_t *s_out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint64_t x = tm_draw(seed, 0, 0, 0);
        s_out[0] = -(int64_t)(x % (uint64_t)L);
    }
}

// window of every sorted edge and whether it is kept
__global__ void k_keep_flags(const int64_t *es_t, int64_t m, const int64_t *s_ptr, int64_t L, uint64_t seed, double p,
                             int64_t *flag, int64_t *win) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    int64_t s = s_ptr[0];
    int64_t j = (es_t[k] - s) / L + 1;
    win[k] = j;
    flag[k] = tm_keep(seed, (uint64_t)j, p) ? 1 : 0;
}

// kept anchors: flag[] holds 0/1 before the scan; scan[] the exclusive sums
__global__ void k_compact(const int64_t *flag01, const int64_t *scan, const int64_t *win, int64_t m, int64_t *apos,
                          int64_t *awin) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m || !flag01[k]) return;
    int64_t i = scan[k];
    apos[i] = k;
    awin[i] = win[k];
}

__global__ void k_copy_i64(const int64_t *src, int64_t *dst, int64_t n) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[k];
}

__global__ void k_slot_flags(const int64_t *awin, const int64_t *nA, int64_t cap, int64_t *sflag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    int64_t n = nA[0];
    sflag[i] = (i < n && (i == 0 || awin[i] != awin[i - 1])) ? 1 : 0;
}

__global__ void k_slot_fill(const int64_t *awin, const int64_t *nA, const int64_t *sflag01, const int64_t *sscan,
                            const int64_t *s_ptr, int64_t L, int32_t *slot, int64_t *slot_win, int64_t *win_end) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nA[0]) return;
    int64_t sl = sscan[i] + sflag01[i] - 1;
    slot[i] = (int32_t)sl;
    int64_t j = awin[i];
    if (sflag01[i]) slot_win[sl] = j;
    win_end[i] = s_ptr[0] + j * L - 1;
}

// kept windows among j = 1..J (diagnostics)
__global__ void k_all_windows(uint64_t seed, int64_t J, double p, int64_t *flag) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (j > J) return;
    flag[j - 1] = tm_keep(seed, (uint64_t)j, p) ? 1 : 0;
}

__global__ void k_list_windows(const int64_t *flag01, const int64_t *scan, int64_t J, int64_t cap, int64_t *ids) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (j > J || !flag01[j - 1]) return;
    int64_t i = scan[j - 1];
    if (i < cap) ids[i] = j;
}

__global__ void k_map_anchors(const int64_t *pos_of, const int64_t *anchor, int64_t n, int64_t m, int64_t *apos,
                              int32_t *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t a = anchor[i];
    if (a < 0 || a >= m) {
        atomicOr(bad, 1);
        apos[i] = 0;
    } else {
        apos[i] = pos_of[a];
    }
}

// r[0] = first sorted edge with time >= lo, r[1] = first with time > hi
__global__ void k_time_range(const int64_t *t, int64_t m, int64_t lo, int64_t hi, int64_t *r) {
    if (blockIdx.x != 0 || threadIdx.x > 1) return;
    const int64_t key = threadIdx.x == 0 ? lo : hi;
    int64_t a = 0, b = m;
    while (a < b) {
        const int64_t mid = a + (b - a) / 2;
        if (threadIdx.x == 0 ? t[mid] < key : t[mid] <= key) a = mid + 1;
        else b = mid;
    }
    r[threadIdx.x] = a;
}

// anchors a0 .. a0 + n - 1 with window end hi
__global__ void k_anchor_range(int64_t a0, int64_t n, int64_t hi, int64_t *pos, int64_t *wend) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    pos[k] = a0 + k;
    wend[k] = hi;
}

tm_status check_graph_motif(const tm_graph *g, const tm_motif *M, int64_t delta, MotifPlan *P) {
    if (!g || !M || delta < 0) return TM_EINVAL;
    return tm_make_plan(M, P);
}

// Anchors of the windows kept by one estimator, on the device.
struct KeptAnchors {
    DevBuf flag, scan, win, apos, awin, sflag, sscan, slot, slot_win, win_end, scal;
    int64_t nA = 0, nslots = 0, s = 0;
};

tm_status select_kept(const tm_graph *g, int64_t L, uint64_t seed, double p, hipStream_t st, KeptAnchors &K) {
    int64_t m = g->m;
    TM_TRY(K.scal.alloc(64));
    int64_t *s_dev = K.scal.as<int64_t>();
    int64_t *nA_dev = s_dev + 1;
    int64_t *ns_dev = s_dev + 2;
    hipLaunchKernelGGL(k_shift, dim3(1), dim3(64), 0, st, seed, L, s_dev);
    TM_HIP(hipGetLastError());
    int64_t cap = m > 0 ? m : 1;
    TM_TRY(K.flag.alloc((size_t)cap * 8));
    TM_TRY(K.scan.alloc((size_t)cap * 8));
    TM_TRY(K.win.alloc((size_t)cap * 8));
    TM_HIP(hipMemsetAsync(nA_dev, 0, 16, st));
    if (m > 0) {
        hipLaunchKernelGGL(k_keep_flags, dim3(tm_blocks(m, TPB)), dim3(TPB), 0, st, g->es_t.as<int64_t>(), m, s_dev,
                           L, seed, p, K.flag.as<int64_t>(), K.win.as<int64_t>());
        TM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_copy_i64, dim3(tm_blocks(m, TPB)), dim3(TPB), 0, st, K.flag.as<int64_t>(),
                           K.scan.as<int64_t>(), m);
        TM_HIP(hipGetLastError());
        TM_TRY(tm_scan_i64(K.scan.as<int64_t>(), m, nA_dev, st));
    }
    TM_HIP(hipMemcpyAsync(&K.nA, nA_dev, 8, hipMemcpyDeviceToHost, st));
    TM_HIP(hipMemcpyAsync(&K.s, s_dev, 8, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    int64_t nA = K.nA, ca = nA > 0 ? nA : 1;
    TM_TRY(K.apos.alloc((size_t)ca * 8));
    TM_TRY(K.awin.alloc((size_t)ca * 8));
    TM_TRY(K.sflag.alloc((size_t)ca * 8));
    TM_TRY(K.sscan.alloc((size_t)ca * 8));
    TM_TRY(K.slot.alloc((size_t)ca * 4));
    TM_TRY(K.slot_win.alloc((size_t)ca * 8));
    TM_TRY(K.win_end.alloc((size_t)ca * 8));
    if (nA > 0) {
        hipLaunchKernelGGL(k_compact, dim3(tm_blocks(m, TPB)), dim3(TPB), 0, st, K.flag.as<int64_t>(),
                           K.scan.as<int64_t>(), K.win.as<int64_t>(), m, K.apos.as<int64_t>(), K.awin.as<int64_t>());
        TM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_slot_flags, dim3(tm_blocks(nA, TPB)), dim3(TPB), 0, st, K.awin.as<int64_t>(), nA_dev, nA,
                           K.sflag.as<int64_t>());
        TM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_copy_i64, dim3(tm_blocks(nA, TPB)), dim3(TPB), 0, st, K.sflag.as<int64_t>(),
                           K.sscan.as<int64_t>(), nA);
        TM_HIP(hipGetLastError());
        TM_TRY(tm_scan_i64(K.sscan.as<int64_t>(), nA, ns_dev, st));
        hipLaunchKernelGGL(k_slot_fill, dim3(tm_blocks(nA, TPB)), dim3(TPB), 0, st, K.awin.as<int64_t>(), nA_dev,
                           K.sflag.as<int64_t>(), K.sscan.as<int64_t>(), s_dev, L, K.slot.as<int32_t>(),
                           K.slot_win.as<int64_t>(), K.win_end.as<int64_t>());
        TM_HIP(hipGetLastError());
        TM_HIP(hipMemcpyAsync(&K.nslots, ns_dev, 8, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
    }
    return TM_OK;
}

// Edge-proportional window probabilities (Sec. 4, equation heuristic_q) for
// shift s of estimator k: window j = 1 .. J gets its edge count from two
// searches of the sorted times, q_j = min(1, r count / m) (a q_j above 1 is
// clamped), and is kept when the uniform of draw (j, k, domain 1) is below
// q_j.  flag[j-1], q[j-1].
__global__ void k_q_windows(const int64_t *es_t, int64_t m, int64_t J, int64_t s, int64_t L, double r,
                            uint64_t seed, uint32_t k, int64_t *flag, double *q, int64_t *range) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (j > J) return;
    const int64_t lo = s + (j - 1) * L, hi = s + j * L - 1;
    int64_t a = 0, b = m;
    while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (es_t[mid] < lo) a = mid + 1;
        else b = mid;
    }
    const int64_t first = a;
    b = m;
    while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (es_t[mid] <= hi) a = mid + 1;
        else b = mid;
    }
    double qj = r * (double)(a - first) / (double)m;
    if (qj > 1.0) qj = 1.0;
    const uint64_t x = tm_draw(seed, (uint64_t)j, k, 1);
    const double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);
    flag[j - 1] = u < qj ? 1 : 0;
    q[j - 1] = qj;
    if (range) {  // the window's edges: sorted positions [first, a)
        range[2 * (j - 1)] = first;
        range[2 * (j - 1) + 1] = a;
    }
}

// kidx[j] = rank of window j among the kept ones (scan: exclusive sums of
// the flags), -1 when not kept; kidx[0] is unused
__global__ void k_q_kidx(const int64_t *flag, const int64_t *scan, int64_t J, int32_t *kidx) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (j == 1) kidx[0] = -1;
    if (j <= J) kidx[j] = flag[j - 1] ? (int32_t)scan[j - 1] : -1;
}

// Time order of one chunk of a host edge stream: bad[0] = 1 when a time is
// below its predecessor (prev: the last time of the previous chunk).
__global__ void k_sorted_chunk(const int64_t *t, int64_t n, int64_t prev, int32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t before = i == 0 ? prev : t[i - 1];
    if (t[i] < before) bad[0] = 1;
}

tm_status check_est_args(const tm_graph *g, int64_t delta, int64_t c, double p, int64_t *L) {
    if (!g || delta < 1 || c < 2 || !(p > 0.0 && p <= 1.0)) return TM_EINVAL;
    if (delta > INT64_MAX / c) return TM_EINVAL;
    *L = c * delta;
    // window ends s + j L - 1 stay below 2^63 for every window of the graph
    if (*L > INT64_MAX / 4 || g->t_span > INT64_MAX - 2 * *L) return TM_EINVAL;
    // the duration histogram has delta + 1 bins
    if (delta > TM_MAX_HIST_DELTA) return TM_EUNSUPPORTED;
    return TM_OK;
}

tm_status fill_info(const tm_graph *g, int64_t L, uint64_t seed, double p, const KeptAnchors &K,
                    const std::vector<uint64_t> &slot_tot, const uint64_t *hist_dev_lo, const uint64_t *hist_dev_hi,
                    int64_t delta, const uint64_t total[2], tm_est_info *info, hipStream_t st) {
    int64_t J = 1 + g->t_span / L + ((g->t_span % L) ? 1 : 0);
    info->shift = K.s;
    info->n_windows = J;
    info->kept_count.lo = total[0];
    info->kept_count.hi = total[1];
    if (J <= ((int64_t)1 << 24)) {
        DevBuf f, sc, ids, tot;
        TM_TRY(f.alloc((size_t)J * 8));
        TM_TRY(sc.alloc((size_t)J * 8));
        TM_TRY(tot.alloc(8));
        int64_t cap = info->cap > 0 ? info->cap : 0;
        TM_TRY(ids.alloc((size_t)(cap > 0 ? cap : 1) * 8));
        hipLaunchKernelGGL(k_all_windows, dim3(tm_blocks(J, TPB)), dim3(TPB), 0, st, seed, J, p, f.as<int64_t>());
        TM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_copy_i64, dim3(tm_blocks(J, TPB)), dim3(TPB), 0, st, f.as<int64_t>(), sc.as<int64_t>(), J);
        TM_HIP(hipGetLastError());
        TM_TRY(tm_scan_i64(sc.as<int64_t>(), J, tot.as<int64_t>(), st));
        hipLaunchKernelGGL(k_list_windows, dim3(tm_blocks(J, TPB)), dim3(TPB), 0, st, f.as<int64_t>(),
                           sc.as<int64_t>(), J, cap, ids.as<int64_t>());
        TM_HIP(hipGetLastError());
        int64_t nk = 0;
        TM_HIP(hipMemcpyAsync(&nk, tot.p, 8, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        info->n_kept = nk;
        int64_t nw = std::min(nk, cap);
        std::vector<int64_t> hids((size_t)(nw > 0 ? nw : 1));
        if (nw > 0) {
            TM_HIP(hipMemcpyAsync(hids.data(), ids.p, (size_t)nw * 8, hipMemcpyDeviceToHost, st));
        }
        std::vector<int64_t> swin((size_t)(K.nslots > 0 ? K.nslots : 1));
        if (K.nslots > 0) {
            TM_HIP(hipMemcpyAsync(swin.data(), K.slot_win.p, (size_t)K.nslots * 8, hipMemcpyDeviceToHost, st));
        }
        TM_HIP(hipStreamSynchronize(st));
        int64_t q = 0;
        for (int64_t i = 0; i < nw; ++i) {
            if (info->kept_ids) info->kept_ids[i] = hids[(size_t)i];
            uint64_t c = 0;
            while (q < K.nslots && swin[(size_t)q] < hids[(size_t)i]) ++q;
            if (q < K.nslots && swin[(size_t)q] == hids[(size_t)i]) c = slot_tot[(size_t)(2 * q)];
            if (info->win_counts) info->win_counts[i] = c;
        }
    } else {
        info->n_kept = -1;
    }
    if (info->hist_lo) {
        TM_HIP(hipMemcpyAsync(info->hist_lo, hist_dev_lo, (size_t)(delta + 1) * 8, hipMemcpyDeviceToHost, st));
    }
    if (info->hist_hi) {
        TM_HIP(hipMemcpyAsync(info->hist_hi, hist_dev_hi, (size_t)(delta + 1) * 8, hipMemcpyDeviceToHost, st));
    }
    TM_HIP(hipStreamSynchronize(st));
    return TM_OK;
}

tm_status estimate_impl(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t c, double p, uint64_t seed,
                        double *estimate, tm_est_info *info, hipStream_t st) {
    MotifPlan P;
    TM_TRY(check_graph_motif(g, M, delta, &P));
    int64_t L;
    TM_TRY(check_est_args(g, delta, c, p, &L));
    if (!estimate) return TM_EINVAL;
    KeptAnchors K;
    TM_TRY(select_kept(g, L, seed, p, st, K));
    if (delta > TM_GENERIC_LDS_DELTA && !(info && (info->hist_lo || info->hist_hi))) {
        // no histogram asked for and none that fits in LDS: the kept
        // instances' fixed-point weights are summed instead
        DevBuf wfx, acc;
        TM_TRY(wfx.alloc((size_t)(delta + 1) * 8));
        const int64_t ns = K.nslots;
        TM_TRY(acc.alloc((size_t)(4 + 2 * (ns > 0 ? ns : 1)) * 8));
        TM_HIP(hipMemsetAsync(acc.p, 0, acc.bytes, st));
        TM_TRY(tm_fx_weights(delta, L, wfx.as<uint64_t>(), st));
        uint64_t *total = acc.as<uint64_t>(), *wsum = total + 2, *slot_tot = total + 4;
        if (K.nA > 0) {
            AnchorSet A{K.nA, K.apos.as<int64_t>(), K.win_end.as<int64_t>(), K.slot.as<int32_t>(), nullptr};
            TM_TRY(tm_count_generic_weighted(g, P, delta, A, total, slot_tot, wfx.as<uint64_t>(), wsum, st));
        }
        uint64_t tw[4];
        std::vector<uint64_t> stot((size_t)(2 * (ns > 0 ? ns : 1)));
        TM_HIP(hipMemcpyAsync(tw, total, 32, hipMemcpyDeviceToHost, st));
        if (ns > 0) TM_HIP(hipMemcpyAsync(stot.data(), slot_tot, (size_t)ns * 16, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        if (info) TM_TRY(fill_info(g, L, seed, p, K, stot, nullptr, nullptr, delta, tw, info, st));
        *estimate = tm_fx_estimate(tw[2], tw[3], p);
        return TM_OK;
    }
    DevBuf hist, acc;
    TM_TRY(hist.alloc((size_t)(delta + 1) * 16));
    int64_t ns = K.nslots;
    TM_TRY(acc.alloc((size_t)(2 + 2 * (ns > 0 ? ns : 1)) * 8 + 64));
    TM_HIP(hipMemsetAsync(hist.p, 0, (size_t)(delta + 1) * 16, st));
    TM_HIP(hipMemsetAsync(acc.p, 0, acc.bytes, st));
    uint64_t *hlo = hist.as<uint64_t>(), *hhi = hlo + (delta + 1);
    uint64_t *total = acc.as<uint64_t>();
    uint64_t *slot_tot = total + 2;
    double *z_dev = (double *)(slot_tot + 2 * (ns > 0 ? ns : 1));
    if (K.nA > 0) {
        AnchorSet A{K.nA, K.apos.as<int64_t>(), K.win_end.as<int64_t>(), K.slot.as<int32_t>(), nullptr};
        TM_TRY(tm_count_generic(g, P, delta, A, total, slot_tot, hlo, hhi, nullptr, nullptr, st));
    }
    TM_TRY(tm_weight(hlo, hhi, delta, L, p, z_dev, st));
    double z = 0;
    uint64_t tot[2];
    std::vector<uint64_t> stot((size_t)(2 * (ns > 0 ? ns : 1)));
    TM_HIP(hipMemcpyAsync(&z, z_dev, 8, hipMemcpyDeviceToHost, st));
    TM_HIP(hipMemcpyAsync(tot, total, 16, hipMemcpyDeviceToHost, st));
    if (ns > 0) TM_HIP(hipMemcpyAsync(stot.data(), slot_tot, (size_t)ns * 16, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    if (info) TM_TRY(fill_info(g, L, seed, p, K, stot, hlo, hhi, delta, tot, info, st));
    *estimate = z;
    return TM_OK;
}

// ---------------------------------------------------------------- sweep path

struct SweepOut {
    uint64_t v[36 * 4];
};

static double u128_scaled(uint64_t lo, uint64_t hi, double scale) {
    double x = (double)hi * 18446744073709551616.0;
    x = x + (double)lo;
    return x * scale;
}

// Runs the 3-edge sweep for the codes in mask; copies the 36 x 4 results and
// (mode 2) the histograms of the requested codes to the host.
// Per host thread, grow-only device workspace of the sweep path: after the
// first calls a query allocates nothing, so queries in flight on different
// threads and streams do not serialise on allocation.
struct SweepWs {
    DevBuf o, h, w, ctr;
};
thread_local SweepWs t_ws;

}  // namespace

void tm_api_release_thread_ws() {
    t_ws.o.release();
    t_ws.h.release();
    t_ws.w.release();
    t_ws.ctr.release();
}

namespace {

tm_status run_sweep(const tm_graph *g, uint64_t mask, int mode, int64_t delta, int windowed, int64_t s, int64_t L,
                    uint64_t seed, double p, SweepOut *out, const std::vector<int> &hist_codes,
                    std::vector<uint64_t> *hist_host, hipStream_t st, const int32_t *kidx = nullptr,
                    uint64_t *win = nullptr) {
    DevBuf &o = t_ws.o, &h = t_ws.h, &w = t_ws.w, &ctr = t_ws.ctr;
    TM_TRY(o.reserve(36 * 4 * 8));
    TM_TRY(ctr.reserve(TM_SWEEP_COUNTER_BYTES));
    if (mode == 2) TM_TRY(h.reserve((size_t)36 * (delta + 1) * 16));
    if (mode == 1) TM_TRY(w.reserve((size_t)(delta + 1) * 8));
    TM_TRY(tm_sweep3(g, mask, mode, delta, windowed, s, L, seed, p, o.as<uint64_t>(), h.as<uint64_t>(),
                     w.as<uint64_t>(), ctr.as<int64_t>(), st, kidx, win, false, true));
    TM_HIP(hipMemcpyAsync(out->v, o.p, sizeof out->v, hipMemcpyDeviceToHost, st));
    if (mode == 2 && hist_host) {
        hist_host->assign(hist_codes.size() * (size_t)(delta + 1) * 2, 0);
        for (size_t k = 0; k < hist_codes.size(); ++k) {
            TM_HIP(hipMemcpyAsync(hist_host->data() + k * (size_t)(delta + 1) * 2,
                                  h.as<uint64_t>() + (size_t)hist_codes[k] * (delta + 1) * 2,
                                  (size_t)(delta + 1) * 16, hipMemcpyDeviceToHost, st));
        }
    }
    TM_HIP(hipStreamSynchronize(st));
    tm_prof_collect();
    return TM_OK;
}

bool all_sweep_codes(int32_t n, const tm_motif *motifs, std::vector<int> *codes, uint64_t *mask) {
    codes->clear();
    *mask = 0;
    for (int32_t i = 0; i < n; ++i) {
        int c = tm_sweep_code_of(&motifs[i]);
        if (c < 0) return false;
        codes->push_back(c);
        *mask |= 1ull << c;
    }
    return n > 0;
}

int64_t host_shift(uint64_t seed, int64_t L) {
    uint64_t x = tm_draw(seed, 0, 0, 0);
    return -(int64_t)(x % (uint64_t)L);
}

// estimates of 3-edge motifs through the sweep: Z = weight / 2^52 / p
tm_status sweep_estimates(const tm_graph *g, int32_t n, const tm_motif *motifs, int64_t delta, int64_t c, double p,
                          uint64_t seed, double *est, tm_u128 *kept, hipStream_t st) {
    int64_t L;
    TM_TRY(check_est_args(g, delta, c, p, &L));
    std::vector<int> codes;
    uint64_t mask;
    if (!all_sweep_codes(n, motifs, &codes, &mask)) return TM_EUNSUPPORTED;
    SweepOut so;
    TM_TRY(run_sweep(g, mask, 1, delta, 1, host_shift(seed, L), L, seed, p, &so, {}, nullptr, st));
    for (int32_t i = 0; i < n; ++i) {
        const uint64_t *v = so.v + 4 * codes[(size_t)i];
        est[i] = u128_scaled(v[2], v[3], 1.0 / 4503599627370496.0) / p;
        if (kept) {
            kept[i].lo = v[0];
            kept[i].hi = v[1];
        }
    }
    return TM_OK;
}

// estimates of a four-edge star (tm_star4_shape) through its own counter:
// Z = weight / 2^52 / p, and its exact count over the kept windows
tm_status star_estimate(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t c, double p, uint64_t seed,
                        double *est, tm_u128 *kept, hipStream_t st) {
    int64_t L;
    TM_TRY(check_est_args(g, delta, c, p, &L));
    uint64_t o[4];
    TM_TRY(tm_star4_run(g, M, 1, delta, 1, host_shift(seed, L), L, seed, p, o, nullptr, st));
    *est = u128_scaled(o[2], o[3], 1.0 / 4503599627370496.0) / p;
    if (kept) {
        kept->lo = o[0];
        kept->hi = o[1];
    }
    return TM_OK;
}

bool is_star4(const tm_motif *M) {
    uint32_t d[4];
    return tm_star4_shape(M, d);
}

static void neumaier_add(double &sum, double &comp, double x) {
    const double t = sum + x;
    if (std::fabs(sum) >= std::fabs(x)) comp += (sum - t) + x;
    else comp += (x - t) + sum;
    sum = t;
}

// Algorithm 1 (Sec. 4) with b shifts and edge-proportional window
// probabilities, for 3-edge motifs through the sweep.  Per shift: window
// flags and q_j on the device, one sweep whose anchors add their exact
// fixed-point sums into their kept window's slot, then on the host
// Z_k = sum over kept windows (ascending j) of Y_{s,j} / q_j with
// Y_{s,j} = weight sum / 2^52; the estimate is the mean of the Z_k.
tm_status estimate_q_impl(const tm_graph *g, int32_t n, const tm_motif *motifs, int64_t delta, int64_t c, double r,
                          int32_t b, uint64_t seed, double *est, tm_q_info *info, hipStream_t st) {
    if (!g || n < 1 || !motifs || !est || !(r > 0.0) || !std::isfinite(r) || b < 1) return TM_EINVAL;
    if (info && info->cap > 0 && (!info->win_k || !info->win_j || !info->win_q || !info->win_y)) return TM_EINVAL;
    int64_t L;
    TM_TRY(check_est_args(g, delta, c, 1.0, &L));
    std::vector<int> codes;
    uint64_t mask;
    // three-edge motifs: one windowed sweep per shift (exact fixed-point
    // sums); otherwise the generic counter per kept window and motif, with
    // its duration histogram weighted in FP64
    const bool sweep = all_sweep_codes(n, motifs, &codes, &mask);
    std::vector<MotifPlan> plans;
    if (!sweep) {
        plans.resize((size_t)n);
        for (int32_t i = 0; i < n; ++i) TM_TRY(check_graph_motif(g, &motifs[i], delta, &plans[(size_t)i]));
        if (delta > TM_MAX_HIST_DELTA) return TM_EUNSUPPORTED;
    }
    const int64_t J = 1 + (g->t_span + L - 1) / L;
    if (J > ((int64_t)1 << 30)) return TM_EUNSUPPORTED;
    std::vector<double> zs(n, 0.0), zc(n, 0.0);
    int64_t n_kept = 0;
    const int64_t cap = info ? info->cap : 0;
    std::vector<int64_t> rk, rj;  // window records, copied to info only on success
    std::vector<double> rq, ry;
    if (g->m > 0) {
        DevBuf flag, scan, qd, kidx, tot, win;
        TM_TRY(flag.alloc((size_t)J * 8));
        TM_TRY(scan.alloc((size_t)J * 8));
        TM_TRY(qd.alloc((size_t)J * 8));
        TM_TRY(kidx.alloc((size_t)(J + 1) * 4));
        TM_TRY(tot.alloc(8));
        std::vector<int64_t> flag_h((size_t)J);
        std::vector<double> q_h((size_t)J);
        std::vector<uint64_t> win_h;
        std::vector<double> y_h;  // Y_{s,j} of each kept window (rows) and motif
        std::vector<int64_t> rng_h;  // generic path: each window's sorted edge range
        DevBuf hist, ydev, ap, we, rng;
        if (!sweep) {
            rng_h.resize((size_t)J * 2);
            TM_TRY(rng.alloc((size_t)J * 16));
            TM_TRY(hist.alloc((size_t)(delta + 1) * 16));
            TM_TRY(ydev.alloc((size_t)n * 8));
        }
        for (int32_t k = 0; k < b; ++k) {
            const int64_t s = -(int64_t)(tm_draw(seed, 0, (uint32_t)k, 0) % (uint64_t)L);
            hipLaunchKernelGGL(k_q_windows, dim3(tm_blocks(J, TPB)), dim3(TPB), 0, st, g->es_t.as<int64_t>(), g->m,
                               J, s, L, r, seed, (uint32_t)k, flag.as<int64_t>(), qd.as<double>(),
                               sweep ? nullptr : rng.as<int64_t>());
            TM_HIP(hipGetLastError());
            TM_HIP(hipMemcpyAsync(scan.p, flag.p, (size_t)J * 8, hipMemcpyDeviceToDevice, st));
            TM_TRY(tm_scan_i64(scan.as<int64_t>(), J, tot.as<int64_t>(), st));
            hipLaunchKernelGGL(k_q_kidx, dim3(tm_blocks(J, TPB)), dim3(TPB), 0, st, flag.as<int64_t>(),
                               scan.as<int64_t>(), J, kidx.as<int32_t>());
            TM_HIP(hipGetLastError());
            int64_t K = 0;
            TM_HIP(hipMemcpyAsync(&K, tot.p, 8, hipMemcpyDeviceToHost, st));
            TM_HIP(hipMemcpyAsync(flag_h.data(), flag.p, (size_t)J * 8, hipMemcpyDeviceToHost, st));
            TM_HIP(hipMemcpyAsync(q_h.data(), qd.p, (size_t)J * 8, hipMemcpyDeviceToHost, st));
            if (!sweep) TM_HIP(hipMemcpyAsync(rng_h.data(), rng.p, (size_t)J * 16, hipMemcpyDeviceToHost, st));
            TM_HIP(hipStreamSynchronize(st));
            std::vector<double> zk(n, 0.0), zkc(n, 0.0);
            if (K > 0) {
                y_h.assign((size_t)K * n, 0.0);
                if (sweep) {
                    TM_TRY(win.reserve((size_t)K * 144 * 8));
                    TM_HIP(hipMemsetAsync(win.p, 0, (size_t)K * 144 * 8, st));
                    SweepOut so;
                    TM_TRY(run_sweep(g, mask, 1, delta, 3, s, L, seed, 1.0, &so, {}, nullptr, st,
                                     kidx.as<int32_t>(), win.as<uint64_t>()));
                    win_h.resize((size_t)K * 144);
                    TM_HIP(hipMemcpyAsync(win_h.data(), win.p, (size_t)K * 144 * 8, hipMemcpyDeviceToHost, st));
                    TM_HIP(hipStreamSynchronize(st));
                    for (int64_t kk = 0; kk < K; ++kk) {
                        for (int32_t i = 0; i < n; ++i) {
                            const uint64_t *v = win_h.data() + (size_t)kk * 144 + 4 * (size_t)codes[(size_t)i];
                            y_h[(size_t)kk * n + i] = u128_scaled(v[2], v[3], 1.0 / 4503599627370496.0);
                        }
                    }
                } else {
                    // anchors of window j: edges with normalised time in
                    // [s + (j-1) L, s + j L - 1], every later edge up to that end
                    int64_t kk = 0;
                    for (int64_t j = 1; j <= J; ++j) {
                        if (!flag_h[(size_t)j - 1]) continue;
                        const int64_t hi = s + j * L - 1;
                        const int64_t a0 = rng_h[2 * ((size_t)j - 1)], a1 = rng_h[2 * ((size_t)j - 1) + 1];
                        const int64_t nA = a1 - a0;
                        if (nA > 0) {
                            std::vector<int64_t> pos((size_t)nA), wend((size_t)nA, hi);
                            for (int64_t x = 0; x < nA; ++x) pos[(size_t)x] = a0 + x;
                            TM_TRY(ap.reserve((size_t)nA * 8));
                            TM_TRY(we.reserve((size_t)nA * 8));
                            TM_HIP(hipMemcpyAsync(ap.p, pos.data(), (size_t)nA * 8, hipMemcpyHostToDevice, st));
                            TM_HIP(hipMemcpyAsync(we.p, wend.data(), (size_t)nA * 8, hipMemcpyHostToDevice, st));
                            const AnchorSet A{nA, ap.as<int64_t>(), we.as<int64_t>(), nullptr, nullptr};
                            uint64_t *hlo = hist.as<uint64_t>(), *hhi = hlo + (delta + 1);
                            for (int32_t i = 0; i < n; ++i) {
                                TM_HIP(hipMemsetAsync(hist.p, 0, (size_t)(delta + 1) * 16, st));
                                TM_TRY(tm_count_generic(g, plans[(size_t)i], delta, A, nullptr, nullptr, hlo, hhi,
                                                        nullptr, nullptr, st));
                                TM_TRY(tm_weight(hlo, hhi, delta, L, 1.0, ydev.as<double>() + i, st));
                            }
                            TM_HIP(hipMemcpyAsync(y_h.data() + (size_t)kk * n, ydev.p, (size_t)n * 8,
                                                  hipMemcpyDeviceToHost, st));
                            // pos and wend are read by the copies above
                            TM_HIP(hipStreamSynchronize(st));
                        }
                        ++kk;
                    }
                }
                int64_t kk = 0;
                for (int64_t j = 1; j <= J; ++j) {
                    if (!flag_h[(size_t)j - 1]) continue;
                    const double q = q_h[(size_t)j - 1];
                    const bool rec = n_kept < cap;
                    for (int32_t i = 0; i < n; ++i) {
                        const double y = y_h[(size_t)kk * n + i];
                        neumaier_add(zk[(size_t)i], zkc[(size_t)i], y / q);
                        if (rec) ry.push_back(y);
                    }
                    if (rec) {
                        rk.push_back(k);
                        rj.push_back(j);
                        rq.push_back(q);
                    }
                    ++kk;
                    ++n_kept;
                }
            }
            for (int32_t i = 0; i < n; ++i) neumaier_add(zs[(size_t)i], zc[(size_t)i], zk[(size_t)i] + zkc[(size_t)i]);
        }
    }
    for (int32_t i = 0; i < n; ++i) est[i] = (zs[(size_t)i] + zc[(size_t)i]) / (double)b;
    if (info) {
        info->n_kept = n_kept;
        for (size_t w = 0; w < rk.size(); ++w) {
            info->win_k[w] = rk[w];
            info->win_j[w] = rj[w];
            info->win_q[w] = rq[w];
            for (int32_t i = 0; i < n; ++i) info->win_y[w * (size_t)n + i] = ry[w * (size_t)n + i];
        }
    }
    return TM_OK;
}

// Algorithm 1 with the windows visited in time order and only one kept
// window's edges on the device at a time (the streaming use of Sec. 4): the
// edges come as host arrays sorted by time; per kept window, its edges are
// loaded as a graph of their own and swept with every anchor (instances of
// that graph are exactly the instances inside the window); the windows'
// exact fixed-point sums add up to the same integers as one in-memory sweep.
tm_status estimate_stream_impl(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t m, int32_t n_nodes,
                               int32_t n, const tm_motif *motifs, int64_t delta, int64_t c, double p, uint64_t seed,
                               double *est, tm_u128 *kept, tm_stream_info *info, hipStream_t st) {
    if (m < 0 || n_nodes <= 0 || (m > 0 && (!src || !dst || !t)) || n < 1 || !motifs || !est) return TM_EINVAL;
    if (delta < 1 || c < 2 || !(p > 0.0 && p <= 1.0) || delta > INT64_MAX / c) return TM_EINVAL;
    const int64_t L = c * delta;
    if (L > INT64_MAX / 4) return TM_EINVAL;
    // three-edge motifs go through the sweep of each window graph; the others
    // through the generic counter, whose duration histograms add up over the
    // windows on the device and are weighted once at the end
    std::vector<int> codes((size_t)n, -1);
    std::vector<MotifPlan> plans((size_t)n);
    std::vector<int32_t> gen;
    uint64_t mask = 0;
    for (int32_t i = 0; i < n; ++i) {
        TM_TRY(tm_make_plan(&motifs[i], &plans[(size_t)i]));
        const int code = tm_sweep_code_of(&motifs[i]);
        if (code >= 0) {
            codes[(size_t)i] = code;
            mask |= 1ull << code;
        } else {
            gen.push_back(i);
        }
    }
    if (!gen.empty() && delta > TM_MAX_HIST_DELTA) return TM_EUNSUPPORTED;
    // generic motifs: duration histograms summed over the windows and weighted
    // at the end, or, above the LDS histogram size, fixed-point weight sums
    // (as tm_estimate does for the same delta)
    const bool wsums = delta > TM_GENERIC_LDS_DELTA;
    const size_t ng = gen.size(), nbins = wsums ? 1 : (size_t)delta + 1;
    DevBuf ghist, gtot, gz, gwfx;
    if (ng > 0) {
        TM_TRY(ghist.alloc(ng * nbins * 16));
        TM_TRY(gtot.alloc(ng * 16));
        TM_TRY(gz.alloc(ng * 8));
        TM_HIP(hipMemsetAsync(ghist.p, 0, ghist.bytes, st));
        TM_HIP(hipMemsetAsync(gtot.p, 0, gtot.bytes, st));
        if (wsums) {
            TM_TRY(gwfx.alloc(((size_t)delta + 1) * 8));
            TM_TRY(tm_fx_weights(delta, L, gwfx.as<uint64_t>(), st));
        }
    }
    // the stream is read on the host: device arrays are refused
    for (const void *ptr : {(const void *)src, (const void *)dst, (const void *)t}) {
        if (!ptr) continue;
        hipPointerAttribute_t attr;
        const hipError_t e = hipPointerGetAttributes(&attr, ptr);
        (void)hipGetLastError();  // plain host memory is unknown to HIP: not an error here
        if (e == hipSuccess && attr.type == hipMemoryTypeDevice) return TM_EINVAL;
    }
    unsigned __int128 wsum[36] = {}, csum[36] = {};
    int64_t J = 0, nk = 0, maxw = 0, peak = 0, s = 0;
    if (m > 0) {
        // time order, checked on the device in bounded chunks
        const int64_t CH = (int64_t)1 << 24;
        DevBuf tc, bad;
        TM_TRY(tc.alloc((size_t)std::min(m, CH) * 8));
        TM_TRY(bad.alloc(4));
        TM_HIP(hipMemsetAsync(bad.p, 0, 4, st));
        int64_t prev = t[0];
        for (int64_t off = 0; off < m; off += CH) {
            const int64_t len = std::min(CH, m - off);
            TM_HIP(hipMemcpyAsync(tc.p, t + off, (size_t)len * 8, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_sorted_chunk, dim3(tm_blocks(len, TPB)), dim3(TPB), 0, st, tc.as<int64_t>(), len,
                               prev, bad.as<int32_t>());
            TM_HIP(hipGetLastError());
            TM_HIP(hipStreamSynchronize(st));  // the chunk buffer is reused
            prev = t[off + len - 1];
        }
        int32_t bad_h = 0;
        TM_HIP(hipMemcpyAsync(&bad_h, bad.p, 4, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        if (bad_h) return TM_EINVAL;
        const int64_t tmin = t[0], tmax = t[m - 1];
        if (tmin < 0 && tmax > INT64_MAX + tmin) return TM_EINVAL;
        const int64_t span = tmax - tmin;
        if (span > INT64_MAX - 2 * L) return TM_EINVAL;
        J = 1 + span / L + ((span % L) ? 1 : 0);
        if (J > ((int64_t)1 << 30)) return TM_EUNSUPPORTED;
        s = host_shift(seed, L);
        // kept windows, on the device
        std::vector<int64_t> ids;
        {
            DevBuf f, sc, di, tot;
            TM_TRY(f.alloc((size_t)J * 8));
            TM_TRY(sc.alloc((size_t)J * 8));
            TM_TRY(di.alloc((size_t)J * 8));
            TM_TRY(tot.alloc(8));
            hipLaunchKernelGGL(k_all_windows, dim3(tm_blocks(J, TPB)), dim3(TPB), 0, st, seed, J, p, f.as<int64_t>());
            TM_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_copy_i64, dim3(tm_blocks(J, TPB)), dim3(TPB), 0, st, f.as<int64_t>(),
                               sc.as<int64_t>(), J);
            TM_HIP(hipGetLastError());
            TM_TRY(tm_scan_i64(sc.as<int64_t>(), J, tot.as<int64_t>(), st));
            hipLaunchKernelGGL(k_list_windows, dim3(tm_blocks(J, TPB)), dim3(TPB), 0, st, f.as<int64_t>(),
                               sc.as<int64_t>(), J, J, di.as<int64_t>());
            TM_HIP(hipGetLastError());
            TM_HIP(hipMemcpyAsync(&nk, tot.p, 8, hipMemcpyDeviceToHost, st));
            TM_HIP(hipStreamSynchronize(st));
            ids.resize((size_t)(nk > 0 ? nk : 1));
            if (nk > 0) TM_HIP(hipMemcpyAsync(ids.data(), di.p, (size_t)nk * 8, hipMemcpyDeviceToHost, st));
            TM_HIP(hipStreamSynchronize(st));
        }
        for (int64_t w = 0; w < nk; ++w) {
            const int64_t j = ids[(size_t)w];
            const int64_t lo = tmin + s + (j - 1) * L, hi = tmin + s + j * L - 1;
            const int64_t a = std::lower_bound(t, t + m, lo) - t;
            const int64_t b = std::upper_bound(t, t + m, hi) - t;
            if (b <= a) continue;  // an empty window holds no instance
            maxw = std::max(maxw, b - a);
            tm_graph *gw = nullptr;
            TM_TRY(tm_load_graph_ex(src + a, dst + a, t + a, b - a, n_nodes, TM_LOAD_NO_EXACT_TABLES, st, &gw));
            SweepOut so;
            tm_status r = TM_OK;
            if (mask) r = run_sweep(gw, mask, 1, delta, 0, 0, L, seed, 1.0, &so, {}, nullptr, st);
            // every anchor of the window graph: its instances are the window's
            const AnchorSet A{gw->m, nullptr, nullptr, nullptr, nullptr};
            for (size_t x = 0; x < ng && r == TM_OK; ++x) {
                uint64_t *hlo = ghist.as<uint64_t>() + x * nbins * 2, *hhi = hlo + nbins;
                r = wsums ? tm_count_generic_weighted(gw, plans[(size_t)gen[x]], delta, A,
                                                      gtot.as<uint64_t>() + 2 * x, nullptr, gwfx.as<uint64_t>(), hlo,
                                                      st)
                          : tm_count_generic(gw, plans[(size_t)gen[x]], delta, A, gtot.as<uint64_t>() + 2 * x,
                                             nullptr, hlo, hhi, nullptr, nullptr, st);
            }
            // the counts read the window graph until they finish
            const hipError_t e = hipStreamSynchronize(st);
            peak = std::max(peak, gw->device_bytes);
            tm_free_graph(gw);
            if (r != TM_OK) return r;
            if (e != hipSuccess) return tm_hip_status(e);
            if (mask) {
                for (int k = 0; k < 36; ++k) {
                    csum[k] += ((unsigned __int128)so.v[4 * k + 1] << 64) | so.v[4 * k];
                    wsum[k] += ((unsigned __int128)so.v[4 * k + 3] << 64) | so.v[4 * k + 2];
                }
            }
        }
    }
    std::vector<double> gz_h(ng);
    std::vector<uint64_t> gtot_h(2 * ng), gw_h(2 * ng);
    if (ng > 0) {
        if (wsums) {
            // per motif, its weight sum is the first two words of its slot
            for (size_t x = 0; x < ng; ++x)
                TM_HIP(hipMemcpyAsync(&gw_h[2 * x], ghist.as<uint64_t>() + x * nbins * 2, 16,
                                      hipMemcpyDeviceToHost, st));
        } else {
            for (size_t x = 0; x < ng; ++x) {
                uint64_t *hlo = ghist.as<uint64_t>() + x * nbins * 2, *hhi = hlo + nbins;
                TM_TRY(tm_weight(hlo, hhi, delta, L, p, gz.as<double>() + x, st));
            }
            TM_HIP(hipMemcpyAsync(gz_h.data(), gz.p, ng * 8, hipMemcpyDeviceToHost, st));
        }
        TM_HIP(hipMemcpyAsync(gtot_h.data(), gtot.p, ng * 16, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        if (wsums)
            for (size_t x = 0; x < ng; ++x) gz_h[x] = tm_fx_estimate(gw_h[2 * x], gw_h[2 * x + 1], p);
    }
    for (size_t x = 0; x < ng; ++x) {
        const int32_t i = gen[x];
        est[i] = gz_h[x];
        if (kept) {
            kept[i].lo = gtot_h[2 * x];
            kept[i].hi = gtot_h[2 * x + 1];
        }
    }
    for (int32_t i = 0; i < n; ++i) {
        const int k = codes[(size_t)i];
        if (k < 0) continue;
        est[i] = u128_scaled((uint64_t)wsum[k], (uint64_t)(wsum[k] >> 64), 1.0 / 4503599627370496.0) / p;
        if (kept) {
            kept[i].lo = (uint64_t)csum[k];
            kept[i].hi = (uint64_t)(csum[k] >> 64);
        }
    }
    if (info) {
        info->shift = s;
        info->n_windows = J;
        info->n_kept = nk;
        info->max_window_edges = maxw;
        info->peak_graph_bytes = peak;
    }
    return TM_OK;
}

tm_status count_exact_impl(const tm_graph *g, const tm_motif *M, int64_t delta, uint64_t *hist_lo_host,
                           uint64_t *hist_hi_host, tm_u128 *out, hipStream_t st) {
    MotifPlan P;
    TM_TRY(check_graph_motif(g, M, delta, &P));
    int code = tm_sweep_code_of(M);
    if (code >= 0 && !hist_lo_host) {
        SweepOut so;
        TM_TRY(run_sweep(g, 1ull << code, 0, delta, 0, 0, 1, 0, 1.0, &so, {}, nullptr, st));
        out->lo = so.v[4 * code];
        out->hi = so.v[4 * code + 1];
        return TM_OK;
    }
    if (!hist_lo_host && is_star4(M)) {
        uint64_t o[4];
        TM_TRY(tm_star4_run(g, M, 0, delta, 0, 0, 1, 0, 1.0, o, nullptr, st));
        out->lo = o[0];
        out->hi = o[1];
        return TM_OK;
    }
    DevBuf acc, hist;
    TM_TRY(acc.alloc(64));
    TM_HIP(hipMemsetAsync(acc.p, 0, 64, st));
    uint64_t *hlo = nullptr, *hhi = nullptr;
    if (hist_lo_host) {
        if (delta > TM_MAX_HIST_DELTA) return TM_EUNSUPPORTED;
        TM_TRY(hist.alloc((size_t)(delta + 1) * 16));
        TM_HIP(hipMemsetAsync(hist.p, 0, hist.bytes, st));
        hlo = hist.as<uint64_t>();
        hhi = hlo + (delta + 1);
    }
    if (g->m > 0) {
        AnchorSet A{g->m, nullptr, nullptr, nullptr, nullptr};
        TM_TRY(tm_count_generic(g, P, delta, A, acc.as<uint64_t>(), nullptr, hlo, hhi, nullptr, nullptr, st));
    }
    uint64_t tot[2];
    TM_HIP(hipMemcpyAsync(tot, acc.p, 16, hipMemcpyDeviceToHost, st));
    if (hlo) {
        TM_HIP(hipMemcpyAsync(hist_lo_host, hlo, (size_t)(delta + 1) * 8, hipMemcpyDeviceToHost, st));
        if (hist_hi_host) TM_HIP(hipMemcpyAsync(hist_hi_host, hhi, (size_t)(delta + 1) * 8, hipMemcpyDeviceToHost, st));
    }
    TM_HIP(hipStreamSynchronize(st));
    out->lo = tot[0];
    out->hi = tot[1];
    return TM_OK;
}

tm_status finish(tm_status s, hipStream_t st) {
    if (s != TM_OK) {
        (void)hipStreamSynchronize(st);
        (void)hipGetLastError();
    }
    tm_prof_collect();
    return s;
}

}  // namespace

extern "C" tm_status tm_count_exact(const tm_graph *g, const tm_motif *M, int64_t delta, tm_u128 *count,
                                    void *hip_stream) {
    if (!count) return TM_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    return finish(count_exact_impl(g, M, delta, nullptr, nullptr, count, st), st);
}

extern "C" tm_status tm_count_exact_i64(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t *count,
                                        void *hip_stream) {
    if (!count) return TM_EINVAL;
    tm_u128 c;
    tm_status s = tm_count_exact(g, M, delta, &c, hip_stream);
    if (s != TM_OK) return s;
    if (c.hi || c.lo > (uint64_t)INT64_MAX) return TM_EOVERFLOW;
    *count = (int64_t)c.lo;
    return TM_OK;
}

extern "C" tm_status tm_count_exact_multi(const tm_graph *g, int32_t n_motifs, const tm_motif *motifs, int64_t delta,
                                          tm_u128 *counts, uint64_t *hist_lo, uint64_t *hist_hi, void *hip_stream) {
    if (!g || n_motifs < 0 || (n_motifs > 0 && (!motifs || !counts)) || delta < 0) return TM_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    MotifPlan P;
    for (int32_t i = 0; i < n_motifs; ++i) TM_TRY(tm_make_plan(&motifs[i], &P));
    std::vector<int> codes;
    uint64_t mask;
    if (all_sweep_codes(n_motifs, motifs, &codes, &mask) && (!hist_lo || delta <= TM_MAX_SWEEP_HIST_DELTA)) {
        auto run = [&]() -> tm_status {
            SweepOut so;
            std::vector<uint64_t> hh;
            TM_TRY(run_sweep(g, mask, hist_lo ? 2 : 0, delta, 0, 0, 1, 0, 1.0, &so, codes, &hh, st));
            for (int32_t i = 0; i < n_motifs; ++i) {
                counts[i].lo = so.v[4 * codes[(size_t)i]];
                counts[i].hi = so.v[4 * codes[(size_t)i] + 1];
                if (hist_lo) {
                    for (int64_t d = 0; d <= delta; ++d) {
                        hist_lo[(int64_t)i * (delta + 1) + d] = hh[((size_t)i * (delta + 1) + d) * 2];
                        if (hist_hi) hist_hi[(int64_t)i * (delta + 1) + d] = hh[((size_t)i * (delta + 1) + d) * 2 + 1];
                    }
                }
            }
            return TM_OK;
        };
        return finish(run(), st);
    }
    for (int32_t i = 0; i < n_motifs; ++i) {
        uint64_t *hl = hist_lo ? hist_lo + (int64_t)i * (delta + 1) : nullptr;
        uint64_t *hh = hist_hi ? hist_hi + (int64_t)i * (delta + 1) : nullptr;
        tm_status s = finish(count_exact_impl(g, &motifs[i], delta, hl, hh, &counts[i], st), st);
        if (s != TM_OK) return s;
    }
    return TM_OK;
}

extern "C" tm_status tm_count_anchors(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t n_anchor,
                                      const int64_t *anchor, const int64_t *win_end, uint64_t *out, void *hip_stream) {
    if (!g || n_anchor < 0 || (n_anchor > 0 && (!anchor || !out)) || delta < 0) return TM_EINVAL;
    MotifPlan P;
    TM_TRY(tm_make_plan(M, &P));
    if (n_anchor == 0) return TM_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    auto run = [&]() -> tm_status {
        DevBuf a, ap, we, o, fl;
        TM_TRY(a.alloc((size_t)n_anchor * 8));
        TM_TRY(ap.alloc((size_t)n_anchor * 8));
        TM_TRY(o.alloc((size_t)n_anchor * 8));
        TM_TRY(fl.alloc(64));
        TM_HIP(hipMemsetAsync(fl.p, 0, 64, st));
        TM_HIP(hipMemcpyAsync(a.p, anchor, (size_t)n_anchor * 8, hipMemcpyHostToDevice, st));
        if (win_end) {
            TM_TRY(we.alloc((size_t)n_anchor * 8));
            TM_HIP(hipMemcpyAsync(we.p, win_end, (size_t)n_anchor * 8, hipMemcpyHostToDevice, st));
        }
        hipLaunchKernelGGL(k_map_anchors, dim3(tm_blocks(n_anchor, TPB)), dim3(TPB), 0, st, g->pos_of.as<int64_t>(),
                           a.as<int64_t>(), n_anchor, g->m, ap.as<int64_t>(), fl.as<int32_t>() + 1);
        TM_HIP(hipGetLastError());
        int32_t bad[2] = {0, 0};
        TM_HIP(hipMemcpyAsync(bad, fl.p, 8, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        if (bad[1]) return TM_EINVAL;
        AnchorSet A{n_anchor, ap.as<int64_t>(), win_end ? we.as<int64_t>() : nullptr, nullptr, nullptr};
        TM_TRY(tm_count_generic(g, P, delta, A, nullptr, nullptr, nullptr, nullptr, o.as<uint64_t>(), fl.as<int32_t>(),
                                st));
        TM_HIP(hipMemcpyAsync(out, o.p, (size_t)n_anchor * 8, hipMemcpyDeviceToHost, st));
        TM_HIP(hipMemcpyAsync(bad, fl.p, 8, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        return bad[0] ? TM_EOVERFLOW : TM_OK;
    };
    return finish(run(), st);
}

extern "C" tm_status tm_estimate(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t c, double p,
                                 uint64_t seed, double *estimate, tm_est_info *info, void *hip_stream) {
    hipStream_t st = (hipStream_t)hip_stream;
    if (!info && g && M && estimate && tm_sweep_code_of(M) >= 0) {
        MotifPlan P;
        TM_TRY(check_graph_motif(g, M, delta, &P));
        return finish(sweep_estimates(g, 1, M, delta, c, p, seed, estimate, nullptr, st), st);
    }
    if (!info && g && M && estimate && is_star4(M)) {
        MotifPlan P;
        TM_TRY(check_graph_motif(g, M, delta, &P));
        return finish(star_estimate(g, M, delta, c, p, seed, estimate, nullptr, st), st);
    }
    return finish(estimate_impl(g, M, delta, c, p, seed, estimate, info, st), st);
}

extern "C" tm_status tm_estimate_q(const tm_graph *g, int32_t n_motifs, const tm_motif *motifs, int64_t delta,
                                   int64_t c, double r, int32_t b, uint64_t seed, double *estimates, tm_q_info *info,
                                   void *hip_stream) {
    hipStream_t st = (hipStream_t)hip_stream;
    return finish(estimate_q_impl(g, n_motifs, motifs, delta, c, r, b, seed, estimates, info, st), st);
}

extern "C" tm_status tm_estimate_stream(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t m,
                                        int32_t n_nodes, int32_t n_motifs, const tm_motif *motifs, int64_t delta,
                                        int64_t c, double p, uint64_t seed, double *estimates, tm_u128 *kept_counts,
                                        tm_stream_info *info, void *hip_stream) {
    hipStream_t st = (hipStream_t)hip_stream;
    return finish(estimate_stream_impl(src, dst, t, m, n_nodes, n_motifs, motifs, delta, c, p, seed, estimates,
                                       kept_counts, info, st),
                  st);
}

extern "C" tm_status tm_estimate_multi(const tm_graph *g, int32_t n_motifs, const tm_motif *motifs, int64_t delta,
                                       int64_t c, double p, uint64_t seed, double *estimates, tm_u128 *kept_counts,
                                       void *hip_stream) {
    if (!g || n_motifs < 0 || (n_motifs > 0 && (!motifs || !estimates))) return TM_EINVAL;
    MotifPlan P;
    for (int32_t i = 0; i < n_motifs; ++i) TM_TRY(tm_make_plan(&motifs[i], &P));
    std::vector<int> codes;
    uint64_t mask;
    if (all_sweep_codes(n_motifs, motifs, &codes, &mask)) {
        hipStream_t st = (hipStream_t)hip_stream;
        return finish(sweep_estimates(g, n_motifs, motifs, delta, c, p, seed, estimates, kept_counts, st), st);
    }
    for (int32_t i = 0; i < n_motifs; ++i) {
        if (is_star4(&motifs[i])) {
            hipStream_t st = (hipStream_t)hip_stream;
            TM_TRY(finish(star_estimate(g, &motifs[i], delta, c, p, seed, &estimates[i],
                                        kept_counts ? &kept_counts[i] : nullptr, st), st));
            continue;
        }
        tm_est_info info;
        memset(&info, 0, sizeof info);
        TM_TRY(tm_estimate(g, &motifs[i], delta, c, p, seed, &estimates[i], kept_counts ? &info : nullptr,
                           hip_stream));
        if (kept_counts) kept_counts[i] = info.kept_count;
    }
    return TM_OK;
}

// ------------------------------------------------ allocation-free estimates

// Device scratch of tm_estimate_multi_noalloc, one copy per GPU, held until
// the process ends: the sweep's 36 x 4 accumulators (144 words), its work
// counters (TM_SWEEP_COUNTER_BYTES: 24 words) and the delta + 1 fixed-point
// weights.  Host code never
// passes the symbol itself to a kernel or a copy: it takes the device
// address of this GPU's copy from hipGetSymbolAddress (noalloc_scratch).
#define TM_NOALLOC_HEAD_WORDS (144 + TM_SWEEP_COUNTER_BYTES / 8)
#define TM_NOALLOC_WORDS ((int64_t)TM_NOALLOC_HEAD_WORDS + TM_NOALLOC_MAX_DELTA + 1)
static __device__ __align__(256) uint64_t scratch[TM_NOALLOC_WORDS];

namespace {

std::mutex g_noalloc_mu;
void *g_noalloc_ptr[64];

// This device's copy of the scratch array, looked up once per device with
// the device current.
tm_status noalloc_scratch(int dev, uint64_t **out) {
    if (dev < 0 || dev >= 64) return TM_EDEVICE;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        int cur = -1;
        TM_HIP(hipGetDevice(&cur));
        if (cur != dev) TM_HIP(hipSetDevice(dev));
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return TM_EDEVICE;
        }
        g_noalloc_ptr[dev] = ptr;
    }
    *out = static_cast<uint64_t *>(g_noalloc_ptr[dev]);
    return TM_OK;
}

// Up to 64 motifs per launch: est[i] = weight sum of code[i] / 2^52 / p and
// kept[i] = its count, the same operations in the same order as the host
// side of tm_estimate_multi (u128 to double, scale by 2^-52, divide by p).
struct NoallocCodes {
    int8_t code[64];
};

__global__ void k_noalloc_final(const uint64_t *out, NoallocCodes c, int32_t n, double p, double *est,
                                tm_u128 *kept) {
    const int i = (int)threadIdx.x;
    if (i >= n) return;
    const uint64_t *v = out + 4 * (int)c.code[i];
    double x = (double)v[3] * 18446744073709551616.0;
    x = x + (double)v[2];
    x = x * (1.0 / 4503599627370496.0);
    est[i] = x / p;
    if (kept) {
        kept[i].lo = v[0];
        kept[i].hi = v[1];
    }
}

}  // namespace

extern "C" tm_status tm_estimate_multi_noalloc(const tm_graph *g, int32_t n_motifs, const tm_motif *motifs,
                                               int64_t delta, int64_t c, double p, uint64_t seed,
                                               double *estimates_dev, tm_u128 *kept_dev, void *hip_stream) {
    if (!g || n_motifs < 1 || !motifs || !estimates_dev) return TM_EINVAL;
    MotifPlan P;
    for (int32_t i = 0; i < n_motifs; ++i) TM_TRY(tm_make_plan(&motifs[i], &P));
    std::vector<int> codes;
    uint64_t mask;
    if (!all_sweep_codes(n_motifs, motifs, &codes, &mask)) return TM_EUNSUPPORTED;
    int64_t L;
    TM_TRY(check_est_args(g, delta, c, p, &L));
    if (delta > TM_NOALLOC_MAX_DELTA) return TM_EUNSUPPORTED;
    uint64_t *base = nullptr;
    TM_TRY(noalloc_scratch(g->device, &base));
    hipStream_t st = (hipStream_t)hip_stream;
    uint64_t *out = base;
    int64_t *ctr = reinterpret_cast<int64_t *>(base + 144);
    uint64_t *wfx = base + TM_NOALLOC_HEAD_WORDS;
    tm_status s = tm_sweep3(g, mask, 1, delta, 1, host_shift(seed, L), L, seed, p, out, nullptr, wfx, ctr, st,
                            nullptr, nullptr, true);
    for (int32_t b = 0; s == TM_OK && b < n_motifs; b += 64) {
        NoallocCodes nc;
        const int32_t k = std::min<int32_t>(64, n_motifs - b);
        for (int32_t i = 0; i < k; ++i) nc.code[i] = (int8_t)codes[(size_t)(b + i)];
        hipLaunchKernelGGL(k_noalloc_final, dim3(1), dim3(64), 0, st, (const uint64_t *)out, nc, k, p,
                           estimates_dev + b, kept_dev ? kept_dev + b : nullptr);
        s = tm_hip_status(hipGetLastError());
    }
    if (s != TM_OK) (void)hipGetLastError();
    return s;
}

extern "C" tm_status tm_estimate_batch(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t c, double p,
                                       int32_t n_seeds, const uint64_t *seeds, int32_t tile, double *estimates,
                                       tm_u128 *kept_counts, void *hip_stream) {
    if (!g || !M || n_seeds < 0 || (n_seeds > 0 && (!seeds || !estimates)) || tile < 0) return TM_EINVAL;
    MotifPlan P;
    TM_TRY(check_graph_motif(g, M, delta, &P));
    int64_t L;
    TM_TRY(check_est_args(g, delta, c, p, &L));
    hipStream_t st = (hipStream_t)hip_stream;
    int code = tm_sweep_code_of(M);
    int64_t J = 1 + g->t_span / L + ((g->t_span % L) ? 1 : 0);
    if (code >= 0 && n_seeds > 0 && (J + 1) * (int64_t)n_seeds <= ((int64_t)1 << 28)) {
        auto run = [&]() -> tm_status {
            int64_t t = tile, b = 8;
            if (t == 0) TM_TRY(tm_batch_tune(g, code, delta, L, p, &t, &b, st));
            return tm_batch_run(g, code, delta, L, p, n_seeds, seeds, t, b, estimates, kept_counts, st);
        };
        return finish(run(), st);
    }
    for (int32_t i = 0; i < n_seeds; ++i) {
        tm_est_info info;
        memset(&info, 0, sizeof info);
        TM_TRY(tm_estimate(g, M, delta, c, p, seeds[i], &estimates[i], kept_counts ? &info : nullptr, hip_stream));
        if (kept_counts) kept_counts[i] = info.kept_count;
    }
    return TM_OK;
}

extern "C" tm_status tm_estimate_mixed(const tm_graph *g, int32_t n, const tm_est_query *q, double *estimates,
                                       tm_u128 *kept_counts, void *hip_stream) {
    return tm_estimate_mixed_ex(g, n, q, estimates, kept_counts, (hipStream_t)hip_stream, true);
}

tm_status tm_estimate_mixed_ex(const tm_graph *g, int32_t n, const tm_est_query *q, double *estimates,
                               tm_u128 *kept_counts, hipStream_t st, bool capture) {
    if (!g || n < 0 || (n > 0 && (!q || !estimates))) return TM_EINVAL;
    std::vector<int32_t> code;
    std::vector<int64_t> delta, L, idx;
    std::vector<double> p;
    std::vector<uint64_t> seed;
    for (int32_t i = 0; i < n; ++i) {
        MotifPlan P;
        TM_TRY(tm_make_plan(&q[i].motif, &P));
        int64_t Li;
        TM_TRY(check_est_args(g, q[i].delta, q[i].c, q[i].p, &Li));
        const int c = tm_sweep_code_of(&q[i].motif);
        if (c < 0) continue;
        code.push_back(c);
        delta.push_back(q[i].delta);
        L.push_back(Li);
        p.push_back(q[i].p);
        seed.push_back(q[i].seed);
        idx.push_back(i);
    }
    // three-edge motifs: one launch for all of them
    const int64_t k = (int64_t)idx.size();
    std::vector<double> est((size_t)(k > 0 ? k : 1));
    std::vector<tm_u128> kept((size_t)(k > 0 ? k : 1));
    tm_status s = tm_batch_mixed(g, k, code.data(), delta.data(), L.data(), p.data(), seed.data(), est.data(),
                                 kept.data(), st, capture);
    if (s != TM_OK) return finish(s, st);
    for (int64_t j = 0; j < k; ++j) {
        estimates[idx[(size_t)j]] = est[(size_t)j];
        if (kept_counts) kept_counts[idx[(size_t)j]] = kept[(size_t)j];
    }
    // the others one after another: four-edge stars through their counter,
    // the rest through the generic counter
    for (int32_t i = 0; i < n; ++i) {
        if (tm_sweep_code_of(&q[i].motif) >= 0) continue;
        if (is_star4(&q[i].motif)) {
            s = finish(star_estimate(g, &q[i].motif, q[i].delta, q[i].c, q[i].p, q[i].seed, &estimates[i],
                                     kept_counts ? &kept_counts[i] : nullptr, st), st);
            if (s != TM_OK) return s;
            continue;
        }
        tm_est_info info;
        memset(&info, 0, sizeof info);
        s = finish(estimate_impl(g, &q[i].motif, q[i].delta, q[i].c, q[i].p, q[i].seed, &estimates[i],
                                 kept_counts ? &info : nullptr, st), st);
        if (s != TM_OK) return s;
        if (kept_counts) kept_counts[i] = info.kept_count;
    }
    return finish(TM_OK, st);
}

extern "C" tm_status tm_batch_release(const tm_graph *g, void *hip_stream) {
    if (!g) return TM_EINVAL;
    // plans may have work in flight on the caller's stream
    TM_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
    tm_batch_release_plans(g);
    return TM_OK;
}

extern "C" tm_status tm_batch_config(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t c, double p,
                                     int32_t *tile, int32_t *blocks_per_cu, void *hip_stream) {
    if (!g || !M || !tile || !blocks_per_cu) return TM_EINVAL;
    MotifPlan P;
    TM_TRY(check_graph_motif(g, M, delta, &P));
    int64_t L;
    TM_TRY(check_est_args(g, delta, c, p, &L));
    int code = tm_sweep_code_of(M);
    if (code < 0) return TM_EUNSUPPORTED;
    hipStream_t st = (hipStream_t)hip_stream;
    int64_t t = 0, b = 0;
    tm_status s = finish(g->m_nl > 0 ? tm_batch_tune(g, code, delta, L, p, &t, &b, st) : TM_OK, st);
    if (s != TM_OK) return s;
    *tile = (int32_t)t;
    *blocks_per_cu = (int32_t)b;
    return TM_OK;
}

extern "C" tm_status tm_count_window(const tm_graph *g, int32_t n_motifs, const tm_motif *motifs, int64_t delta,
                                     int64_t t_lo, int64_t t_hi, tm_u128 *counts, void *hip_stream) {
    if (!g || n_motifs < 0 || (n_motifs > 0 && (!motifs || !counts)) || delta < 0 || t_lo > t_hi) return TM_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    MotifPlan P;
    for (int32_t i = 0; i < n_motifs; ++i) TM_TRY(tm_make_plan(&motifs[i], &P));
    // normalised window bounds, clamped to the graph's time range
    int64_t lo = (t_lo <= g->t_min) ? 0 : t_lo - g->t_min;
    int64_t hi;
    if (t_hi < g->t_min) {
        for (int32_t i = 0; i < n_motifs; ++i) counts[i].lo = counts[i].hi = 0;
        return TM_OK;
    }
    hi = (t_hi - g->t_min > g->t_span) ? g->t_span : t_hi - g->t_min;
    std::vector<int> codes;
    uint64_t mask;
    if (all_sweep_codes(n_motifs, motifs, &codes, &mask)) {
        auto run = [&]() -> tm_status {
            SweepOut so;
            TM_TRY(run_sweep(g, mask, 0, delta, 2, lo, hi, 0, 1.0, &so, {}, nullptr, st));
            for (int32_t i = 0; i < n_motifs; ++i) {
                counts[i].lo = so.v[4 * codes[(size_t)i]];
                counts[i].hi = so.v[4 * codes[(size_t)i] + 1];
            }
            return TM_OK;
        };
        return finish(run(), st);
    }
    // other motifs: generic counter over the window's anchors, the window's
    // range of the sorted times found on the device
    auto run = [&]() -> tm_status {
        int64_t a[2] = {0, 0};
        if (g->m > 0) {
            DevBuf r;
            TM_TRY(r.alloc(16));
            hipLaunchKernelGGL(k_time_range, dim3(1), dim3(64), 0, st, g->es_t.as<int64_t>(), g->m, lo, hi,
                               r.as<int64_t>());
            TM_HIP(hipGetLastError());
            TM_HIP(hipMemcpyAsync(a, r.p, 16, hipMemcpyDeviceToHost, st));
            TM_HIP(hipStreamSynchronize(st));
        }
        const int64_t a0 = a[0], nA = a[1] > a[0] ? a[1] - a[0] : 0;
        DevBuf ap, we;
        if (nA > 0) {
            TM_TRY(ap.alloc((size_t)nA * 8));
            TM_TRY(we.alloc((size_t)nA * 8));
            hipLaunchKernelGGL(k_anchor_range, dim3(tm_blocks(nA, TPB)), dim3(TPB), 0, st, a0, nA, hi,
                               ap.as<int64_t>(), we.as<int64_t>());
            TM_HIP(hipGetLastError());
        }
        for (int32_t i = 0; i < n_motifs; ++i) {
            TM_TRY(tm_make_plan(&motifs[i], &P));
            if (is_star4(&motifs[i])) {
                uint64_t o[4];
                TM_TRY(tm_star4_run(g, &motifs[i], 0, delta, 2, lo, hi, 0, 1.0, o, nullptr, st));
                counts[i].lo = o[0];
                counts[i].hi = o[1];
                continue;
            }
            DevBuf acc;
            TM_TRY(acc.alloc(64));
            TM_HIP(hipMemsetAsync(acc.p, 0, 64, st));
            if (nA > 0) {
                AnchorSet A{nA, ap.as<int64_t>(), we.as<int64_t>(), nullptr, nullptr};
                TM_TRY(tm_count_generic(g, P, delta, A, acc.as<uint64_t>(), nullptr, nullptr, nullptr, nullptr, nullptr,
                                        st));
            }
            uint64_t tot[2];
            TM_HIP(hipMemcpyAsync(tot, acc.p, 16, hipMemcpyDeviceToHost, st));
            TM_HIP(hipStreamSynchronize(st));
            counts[i].lo = tot[0];
            counts[i].hi = tot[1];
        }
        return TM_OK;
    };
    return finish(run(), st);
}

extern "C" tm_status tm_profile_enable(int32_t on) {
    ProfState &P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    if (on < 0 || on > 2) return TM_EINVAL;
    P.on = on != 0;
    P.serial = on == 2;
    return TM_OK;
}

extern "C" tm_status tm_profile_reset(void) {
    tm_prof_collect();
    ProfState &P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.total.clear();
    return TM_OK;
}

extern "C" tm_status tm_profile_read(const char *kernel, double *total_ms, int64_t *launches) {
    if (!kernel || !total_ms || !launches) return TM_EINVAL;
    tm_prof_collect();
    ProfState &P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.total.find(kernel);
    if (it == P.total.end()) {
        *total_ms = 0.0;
        *launches = 0;
    } else {
        *total_ms = it->second.first;
        *launches = it->second.second;
    }
    return TM_OK;
}

extern "C" tm_status tm_sweep_census(const tm_graph *g, int64_t delta, tm_census *out, void *hip_stream) {
    if (!g || delta < 0 || !out) return TM_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    tm_census c;
    c.anchors = 2 * g->m_nl;
    c.tri_anchors = g->n_hi;
    tm_status s = finish(tm_sweep_census_impl(g, delta, 0, 0, 0.0, 0, &c, st), st);
    if (s == TM_OK) *out = c;
    return s;
}

extern "C" tm_status tm_sweep_census_est(const tm_graph *g, int64_t delta, int64_t c, double p, uint64_t seed,
                                         tm_census *out, void *hip_stream) {
    if (!g || !out) return TM_EINVAL;
    int64_t L;
    TM_TRY(check_est_args(g, delta, c, p, &L));
    hipStream_t st = (hipStream_t)hip_stream;
    tm_census r;
    tm_status s = finish(tm_sweep_census_impl(g, delta, host_shift(seed, L), L, p, seed, &r, st), st);
    if (s == TM_OK) *out = r;
    return s;
}

extern "C" tm_status tm_tri_static_census(const tm_graph *g, int64_t delta, int64_t c, double p, uint64_t seed,
                                          tm_tri_census *out, void *hip_stream) {
    if (!g || !out) return TM_EINVAL;
    int64_t L;
    TM_TRY(check_est_args(g, delta, c, p, &L));
    hipStream_t st = (hipStream_t)hip_stream;
    tm_tri_census r;
    tm_status s = finish(tm_tri_static_census_impl(g, delta, host_shift(seed, L), L, seed, p, &r, st), st);
    if (s == TM_OK) *out = r;
    return s;
}

extern "C" const char *tm_strerror(tm_status s) {
    switch (s) {
        case TM_OK: return "ok";
        case TM_EINVAL: return "invalid argument";
        case TM_EUNSUPPORTED: return "unsupported motif";
        case TM_ENOMEM: return "out of memory";
        case TM_EBUDGET: return "over memory budget";
        case TM_EOVERFLOW: return "count overflows the requested width";
        case TM_EDEVICE: return "HIP device error";
    }
    return "unknown status";
}

extern "C" const char *tm_version(void) { return "tm 0.1 gfx950"; }
