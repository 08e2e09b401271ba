// Internal declarations shared by the HIP sources of libtm (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <map>
#include <shared_mutex>
#include <vector>

#include "tm.h"

#define TM_WAVE 64

// Work counters of the three-edge sweep: one per XCD for each of its three
// kernels (the claim ranges of SweepArgs::parts).
#define TM_SWEEP_PARTS 8
#define TM_SWEEP_COUNTER_BYTES (3 * TM_SWEEP_PARTS * 8)

// Largest delta for which a duration histogram (delta + 1 bins) is built.
#define TM_MAX_HIST_DELTA ((int64_t)1 << 26)

// Host-side status propagation.
#define TM_TRY(expr)                          \
    do {                                      \
        tm_status _s = (expr);                \
        if (_s != TM_OK) return _s;           \
    } while (0)

static inline tm_status tm_hip_status(hipError_t e) {
    if (e == hipSuccess) return TM_OK;
    if (e == hipErrorOutOfMemory) return TM_ENOMEM;
    return TM_EDEVICE;
}

#define TM_HIP(expr) TM_TRY(tm_hip_status(expr))

// Device blocks that graph loads on this host thread freed, kept for the
// next load: hipMalloc and hipFree cost 0.1-0.2 ms each and a load makes
// about forty of each for its temporaries.  Only allocations and frees made
// while a load runs (LoadCacheScope) go through the cache, which keeps at
// most TM_LOAD_CACHE_BYTES and gives its blocks back to the device when an
// allocation runs out of memory.
constexpr size_t TM_LOAD_CACHE_BYTES = (size_t)2 << 30;

// hipFree performs an implicit device-wide synchronisation, which a stream
// that another thread is capturing into a hipGraph does not allow.  The
// library's frees and device synchronisations therefore hold this lock
// shared, and its captures (BeginCapture .. EndCapture) hold it exclusively,
// so that none of its frees overlaps one of its captures.
inline std::shared_mutex &tm_capture_lock() {
    static std::shared_mutex m;
    return m;
}

// The other runtime calls that may synchronise or take the device's
// allocator (device allocation, graph instantiation, stream and event
// creation) hold the lock shared too: on this runtime a free made by one
// thread while another captures broke the process, and an allocation is the
// same kind of call.  Never called while the thread holds the lock
// exclusively (captures only enqueue kernels, copies and event waits).
template <class F>
inline hipError_t tm_locked_call(F &&f) {
    std::shared_lock<std::shared_mutex> lk(tm_capture_lock());
    return f();
}

// Device bytes held by the calling host thread: what its DevBufs allocated
// minus what they freed (blocks kept by the load cache count as held), and
// the high-water mark since the caller last set peak = live.  The query
// server charges each batch's workspace against its budget and checks the
// charge against this measurement.
struct DevTally {
    int64_t live = 0, peak = 0;
    void add(int64_t b) {
        live += b;
        if (live > peak) peak = live;
    }
};
inline thread_local DevTally t_dev_tally;

struct LoadCache {
    std::multimap<size_t, void *> blocks;  // block size -> block
    size_t bytes = 0;
    size_t limit = TM_LOAD_CACHE_BYTES;    // 0: keep nothing (server slot threads)
    bool active = false;
    void clear() {
        if (blocks.empty()) return;
        std::shared_lock<std::shared_mutex> lk(tm_capture_lock());
        for (auto &kv : blocks) {
            (void)hipFree(kv.second);
            t_dev_tally.add(-(int64_t)kv.first);
        }
        blocks.clear();
        bytes = 0;
    }
    ~LoadCache() { clear(); }
};
inline thread_local LoadCache t_load_cache;

struct LoadCacheScope {
    bool prev;
    LoadCacheScope() : prev(t_load_cache.active) { t_load_cache.active = true; }
    LoadCacheScope(const LoadCacheScope &) = delete;
    LoadCacheScope &operator=(const LoadCacheScope &) = delete;
    ~LoadCacheScope() { t_load_cache.active = prev; }
};

// Owned device allocation (freed on destruction).  bytes is the size asked
// for; a block taken from the load cache can be larger (cap).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    size_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            LoadCache &C = t_load_cache;
            bool kept = false;
            if (C.active && C.bytes + cap <= C.limit) {
                try {
                    C.blocks.emplace(cap, p);
                    C.bytes += cap;
                    kept = true;
                } catch (...) {
                }
            }
            if (!kept) {
                std::shared_lock<std::shared_mutex> lk(tm_capture_lock());
                (void)hipFree(p);
                t_dev_tally.add(-(int64_t)cap);
            }
        }
        p = nullptr;
        bytes = 0;
        cap = 0;
    }
    tm_status alloc(size_t nbytes) {
        release();
        if (nbytes == 0) nbytes = 256;
        LoadCache &C = t_load_cache;
        if (C.active) {
            // a cached block of at least the size and at most a quarter more
            // (graph buffers come from here too; a reload asks the same sizes)
            auto it = C.blocks.lower_bound(nbytes);
            if (it != C.blocks.end() && it->first <= nbytes + nbytes / 4) {
                p = it->second;
                cap = it->first;
                bytes = nbytes;
                C.bytes -= it->first;
                C.blocks.erase(it);
                return TM_OK;
            }
        }
        hipError_t e = tm_locked_call([&] { return hipMalloc(&p, nbytes); });
        if (e == hipErrorOutOfMemory && !C.blocks.empty()) {
            (void)hipGetLastError();
            C.clear();
            e = tm_locked_call([&] { return hipMalloc(&p, nbytes); });
        }
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return e == hipErrorOutOfMemory ? TM_ENOMEM : TM_EDEVICE;
        }
        bytes = nbytes;
        cap = nbytes;
        t_dev_tally.add((int64_t)nbytes);
        return TM_OK;
    }
    // grow-only reuse
    tm_status reserve(size_t nbytes) {
        if (p && bytes >= nbytes) return TM_OK;
        return alloc(nbytes);
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Device-resident, immutable temporal graph.
//
// Times are normalised (t' = t - t_min, the origin of Algorithm 1) and kept
// as int64.  Self-loop edges stay in the time-sorted edge array (they are
// edges of the graph and count towards window sizes) but are left out of
// every incidence list, since no motif edge can map onto them.
struct tm_graph {
    int device = 0;
    int64_t m = 0, n = 0;
    int64_t t_min = 0, t_span = 0;
    int64_t m_nl = 0;   // edges that are not self-loops
    int64_t S = 0;      // distinct directed pairs (u != v)

    // time-sorted edges (ties in input order)
    DevBuf es_src, es_dst, es_t;   // int32, int32, int64 [m]
    DevBuf pos_of;                 // int64 [m]: input index -> sorted position

    // per-node time-sorted out- and in-lists (non-self-loop edges)
    DevBuf out_off, out_nbr, out_t;  // int64[n+1], int32[m_nl], int64[m_nl]
    DevBuf in_off, in_nbr, in_t;

    // combined incidence lists: every non-self-loop edge appears in the list
    // of its source (direction bit 0) and of its destination (bit 1), times
    // ascending within a list
    DevBuf inc_off;  // int64[n+1]
    DevBuf inc_nd;   // uint32[2 m_nl]: other endpoint | (dir << 31)
    DevBuf inc_t;    // int64[2 m_nl]
    DevBuf inc_twin; // uint32[2 m_nl]: position of the same edge in its other endpoint's list
    // ranked sublists: the entries of each combined list whose other endpoint
    // ranks above the list's owner (rank = (incidence-list length, node id)),
    // in the same time order
    int64_t n_hi = 0;
    DevBuf hi_off;   // int64[n+1]
    DevBuf hi_nd;    // uint32[n_hi]
    DevBuf hi_t;     // int64[n_hi]

    // unordered pairs {a < b}: one time-sorted timeline per pair holding the
    // edges of both directions; entry e carries its time and the number of
    // a -> b edges among the pair's earlier entries, and a sentinel entry
    // after the last one carries the pair's a -> b total
    int64_t U = 0;   // distinct unordered pairs
    DevBuf up_ent;   // PairEnt[m_nl + U]
    // unordered pair hash (open addressing, linear probing): slot = key
    // (min << 32 | max, ~0 when empty), the unordered pair id and a copy of
    // the pair's metadata
    DevBuf ph_slot;  // PairSlot[ph_cap]
    int64_t ph_cap = 0;
    // per unordered pair time buckets: bucket b of pair p covers times
    // [t_first + b 2^shift, t_first + (b+1) 2^shift), the widest buckets
    // with at most TM_PAIR_BUCKET_DENSITY per entry; pbk holds, per bucket, the
    // index (relative to the pair's first entry) of its first entry and the
    // a -> b edges before it, plus a sentinel bucket (size, a -> b total), so
    // that a time in an empty bucket is answered without reading entries
    DevBuf pmeta;    // PairMeta[U]
    DevBuf pbk;      // PairBucket[sum (nb + 1)]

    // exact-count tables (tm_exact.hip): per pair entry and endpoint view,
    // global prefix sums of six counts split by the entry's direction, so
    // that the exact 2-node and star counts of an anchor are range sums
    int want_ex = 1;    // build them at load (TM_LOAD_NO_EXACT_TABLES clears it)
    int has_ex = 0;
    int64_t ex_S = 0;   // pair entry slots (m_nl + U, sentinels included)
    DevBuf ex_c0x;      // int64[2 m_nl + 1]: direction-0 entries before each list position (global)
    DevBuf ex_rows;     // uint64[2][ex_S][12]

    // four-edge stars (tm_star4.hip): per incidence entry, the rank of its
    // other endpoint among the owner's heaviest neighbours, built on first use
    DevBuf s4_rank;   // uint8[2 m_nl]

    // static triangles (tm_tri_static.hip), built on first use by a weighted
    // triangle estimate: nodes ascending and the pair opposite each
    int st_state = 0;   // 0 not built, 1 built, 2 not kept (too many)
    int64_t st_ntri = 0;
    DevBuf st_tri;      // {uint32 u[3]; int32 q[3]}[st_ntri]

    // reusable per-graph workspace for queries
    DevBuf ws;
    int64_t device_bytes = 0;
};

// One cache line per slot: the key and, inline, what a lookup in the pair
// needs (a copy of its PairMeta and its size), so that finding a pair and
// reading its metadata is one access.
// Lookups read the first 48 bytes as three 16-byte vectors, so the field
// order and offsets are fixed (static_asserts below).
struct __attribute__((aligned(64))) PairSlot {
    uint64_t key;
    int64_t t0, base, boff;  // as in PairMeta
    int32_t id;              // unordered pair id, -1 when empty
    int32_t shift, nb;       // as in PairMeta
    uint32_t n;              // number of entries
};
static_assert(offsetof(PairSlot, t0) == 8 && offsetof(PairSlot, base) == 16 && offsetof(PairSlot, boff) == 24 &&
                  offsetof(PairSlot, id) == 32 && offsetof(PairSlot, shift) == 36 && offsetof(PairSlot, nb) == 40 &&
                  offsetof(PairSlot, n) == 44 && sizeof(PairSlot) == 64,
              "PairSlot layout is read as three 16-byte vectors");

constexpr int64_t TM_PAIR_BUCKET_DENSITY = 8;

struct __attribute__((aligned(8))) PairBucket {
    uint32_t idx;  // first entry at or after the bucket's start (relative)
    uint32_t c0;   // a -> b edges before that entry
};
static_assert(sizeof(PairBucket) == 8, "two adjacent buckets are read as one 16-byte load");

struct __attribute__((aligned(16))) PairEnt {
    int64_t t;     // time (LLONG_MAX in the sentinel)
    int64_t c0;    // a -> b edges among the pair's earlier entries
};

struct __attribute__((aligned(32))) PairMeta {
    int64_t t0;    // time of the pair's first entry
    int64_t base;  // index of its first entry in up_ent
    int64_t boff;  // its first bucket in pbk
    int32_t shift; // bucket width 2^shift
    int32_t nb;    // buckets (pbk[boff + nb] = sentinel: size, a -> b total)
};

// Plain-pointer view of a graph for kernels.
struct DevGraph {
    int64_t m, n, m_nl, S;
    const int32_t *es_src, *es_dst;
    const int64_t *es_t;
    const int64_t *out_off; const int32_t *out_nbr; const int64_t *out_t;
    const int64_t *in_off; const int32_t *in_nbr; const int64_t *in_t;
    const int64_t *inc_off; const uint32_t *inc_nd; const int64_t *inc_t; const uint32_t *inc_twin;
    int64_t n_hi; const int64_t *hi_off; const uint32_t *hi_nd; const int64_t *hi_t;
    const PairSlot *ph_slot; int64_t ph_cap;
    const PairMeta *pmeta; const PairBucket *pbk;
    const PairEnt *up_ent;
    int has_ex; int64_t ex_S; const int64_t *ex_c0x; const uint64_t *ex_rows;
};

__device__ inline uint64_t tm_pair_hash(uint64_t key, int64_t cap) {
    return (key * 0x9E3779B97F4A7C15ull) >> (64 - __builtin_ctzll((unsigned long long)cap));
}

DevGraph dev_view(const tm_graph *g);

// Builds the exact-count tables of a loaded graph (ent_nl: edge index of
// each pair entry slot, ~0 for sentinels; inc_pos: list position of each
// edge's source (2k) and destination (2k + 1) entry; nl_pos: edge index ->
// time-sorted position).  Leaves has_ex = 0 when they do not fit in a
// quarter of the free device memory.
tm_status tm_build_exact_tables(tm_graph *g, const uint32_t *ent_nl, const uint32_t *inc_pos, const int64_t *nl_pos,
                                hipStream_t st);

// ------------------------------------------------------------ primitives

// Grow-only device workspaces the query paths keep per host thread (sweep
// accumulators, claim orders, scan block sums, generic-counter items), and
// the sizes they reach: the query server frees them after every batch, so
// that a batch's device memory is exactly what it was charged.
void tm_api_release_thread_ws();
void tm_sweep_release_thread_ws();
void tm_prims_release_thread_ws();
void tm_generic_release_thread_ws();
void tm_batch_release_thread_ws();
void tm_star4_release_thread_ws();
void tm_tri_static_release_thread_ws();
inline void tm_release_thread_ws() {
    tm_api_release_thread_ws();
    tm_sweep_release_thread_ws();
    tm_prims_release_thread_ws();
    tm_generic_release_thread_ws();
    tm_batch_release_thread_ws();
    tm_star4_release_thread_ws();
    tm_tri_static_release_thread_ws();
    t_load_cache.clear();
}
int64_t tm_scan_ws_bytes(int64_t n);           // block sums of a scan of n values
int64_t tm_radix_sort_bytes(int64_t n);        // temporaries of a radix sort of n pairs
int64_t tm_tri_order_bytes(const tm_graph *g); // the exact triangle sweep's claim order
int64_t tm_generic_bytes(int64_t n_anchors, int len);  // the generic counter's items

// Exclusive prefix sum of n int64 values, in place; *total (nullable, device)
// receives the sum.  Asynchronous on st; its block sums live in a per-thread
// workspace that grows on demand (a host thread scans on one stream at a time).
tm_status tm_scan_i64(int64_t *d, int64_t n, int64_t *d_total, hipStream_t st);

// Stable LSD radix sort of (key, val) pairs by the low `bits` bits of key.
// keys/vals are sorted in place (ping-pong buffers allocated internally).
tm_status tm_radix_sort(uint64_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t st);

// Number of significant bits of x (0 for x == 0).
static inline int tm_bitlen(uint64_t x) {
    int b = 0;
    while (x) { ++b; x >>= 1; }
    return b;
}

static inline unsigned tm_blocks(int64_t n, int per_block) {
    int64_t b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// ------------------------------------------------------------ 128-bit atomics

__device__ inline void tm_atomic_add_u128(uint64_t *lo, uint64_t *hi, uint64_t vlo, uint64_t vhi) {
    if (vlo) {
        unsigned long long old = atomicAdd((unsigned long long *)lo, (unsigned long long)vlo);
        if (old + vlo < old) vhi += 1;
    }
    if (vhi) atomicAdd((unsigned long long *)hi, (unsigned long long)vhi);
}

// 128-bit add of (blo, bhi) into (alo, ahi)
__device__ __host__ inline void tm_add_u128(uint64_t &alo, uint64_t &ahi, uint64_t blo, uint64_t bhi) {
    uint64_t s = alo + blo;
    ahi += bhi + (s < alo ? 1 : 0);
    alo = s;
}

// ------------------------------------------------------------ motif plans

// Level r >= 1 of a motif scans one list, chosen by which endpoints of motif
// edge r were bound by edges 0..r-1.
enum : int32_t { LV_PAIR = 0, LV_OUT = 1, LV_IN = 2 };

struct MotifPlan {
    int32_t l, k;
    int32_t kind[4];
    int32_t u[4], v[4];
};

// Validates a motif (canonical labels, no self-loop, prefix-connected, l<=4)
// and builds its plan.
tm_status tm_make_plan(const tm_motif *M, MotifPlan *P);

// ------------------------------------------------------------ anchors

// Anchor description for the counters: either every sorted edge (exact) or a
// compacted list of sorted positions (kept windows) with a window end time.
struct AnchorSet {
    int64_t n;              // number of anchors (host-known upper bound if dev_n)
    const int64_t *pos;     // sorted positions, or nullptr for 0..n-1
    const int64_t *win_end; // per anchor window end (nullable: +inf)
    const int32_t *slot;    // per anchor output slot (nullable)
    const int64_t *dev_n;   // device-side anchor count (nullable)
};

// Generic counter (any supported motif).  Adds into total (2 x u64),
// per-slot totals (2 x u64 per slot, nullable), histogram (delta+1 bins,
// lo/hi, nullable), per-anchor outputs (u64, nullable, +overflow flag).
tm_status tm_count_generic(const tm_graph *g, const MotifPlan &P, int64_t delta, const AnchorSet &A,
                           uint64_t *total, uint64_t *slot_tot, uint64_t *hist_lo,
                           uint64_t *hist_hi, uint64_t *per_anchor, int32_t *flag,
                           hipStream_t st);

// FP64 weighting of a duration histogram (single work-item, ascending order,
// Neumaier compensation): out[0] = (1/p) sum N(d) L/(L-d).
tm_status tm_weight(const uint64_t *hist_lo, const uint64_t *hist_hi, int64_t delta, int64_t L,
                    double p, double *out, hipStream_t st);

// Largest delta whose duration histogram the generic counter keeps in LDS;
// above it the estimate paths sum fixed-point weights instead
// (tm_count_generic_weighted) rather than building a histogram in global
// memory with one atomic add per instance.
constexpr int64_t TM_GENERIC_LDS_DELTA = 8191;

// The generic counter's totals (as tm_count_generic, no histogram) and the
// sum of the instances' fixed-point weights wfx[t_l - t_1] (delta + 1 of
// them, tm_fx_weights) added to wsum[0] (low word) and wsum[1] (high word).
tm_status tm_count_generic_weighted(const tm_graph *g, const MotifPlan &P, int64_t delta, const AnchorSet &A,
                                    uint64_t *total, uint64_t *slot_tot, const uint64_t *wfx, uint64_t *wsum,
                                    hipStream_t st);

// wfx[d] = round(2^52 L / (L - d)) for d = 0 .. delta (L >= 2 delta): the
// estimator's weight 1 / (1 - d / L) in 52-bit fixed point, the same table as
// the sweeps'.
tm_status tm_fx_weights(int64_t delta, int64_t L, uint64_t *wfx, hipStream_t st);

// An estimate from a 128-bit sum of fixed-point weights: (hi 2^64 + lo) 2^-52 / p,
// in the same operation order as the sweep paths.
inline double tm_fx_estimate(uint64_t lo, uint64_t hi, double p) {
    double x = (double)hi * 18446744073709551616.0;
    x = x + (double)lo;
    x = x * (1.0 / 4503599627370496.0);
    return x / p;
}

// ------------------------------------------------------------ 3-edge sweep

// The 36 motifs with three edges on two or three nodes, indexed 0..35 by the
// sweep counter (canonical labels).
void tm_sweep_code_motif(int code, tm_motif *M);
int tm_sweep_code_of(const tm_motif *M);  // -1 when M is not one of them

// Sweep counter.  mode 0: counts; 1: counts and fixed-point weighted sums
// (weights round(2^52 L / (L - Delta)) written to wfx_dev); 2: counts and
// duration histograms (hist_dev: 36 x (delta+1) x {lo, hi}).  out_dev:
// 36 x {count lo, count hi, weight lo, weight hi}.  windowed: 0 every anchor;
// 1 anchors in windows kept by (seed, p) under shift s and window length L;
// 2 anchors in the one window [s, L]; 3 anchors in windows j (shift s,
// length L) with kidx_dev[j] >= 0, whose sums go to the window's own slot
// win_dev + 144 kidx_dev[j] (same layout as out_dev) instead of out_dev.
// counter_dev: 8 int64 work-queue heads.  single_stream: run the pass's
// kernels one after another on st instead of forking them onto the calling
// thread's side streams (which are created on first use).  Accumulators and
// counters are cleared by a kernel, not a memset.  static_tri: in mode 1
// over kept windows (windowed 1 or 3), count the triangle codes over the
// static triangles
// (tm_tri_static_weight, which allocates and synchronises st) instead of the
// incidence lists.  Allocates nothing in modes 1 and 2 without static_tri;
// the exact triangle sweep of mode 0 sorts its claim order in
// a per-thread workspace.
tm_status tm_sweep3(const tm_graph *g, uint64_t code_mask, int mode, int64_t delta, int windowed, int64_t s,
                    int64_t L, uint64_t seed, double p, uint64_t *out_dev, uint64_t *hist_dev, uint64_t *wfx_dev,
                    int64_t *counter_dev, hipStream_t st, const int32_t *kidx_dev = nullptr,
                    uint64_t *win_dev = nullptr, bool single_stream = false, bool static_tri = false);

// Weighted triangle sums (codes 20..27 of out, added to) of the kept windows
// of (s, L, seed, p) over the graph's static triangles, built on first use;
// with kidx (window j kept when kidx[j] >= 0, j = 1 .. the last window of the
// graph) the sums of each kept window go to its own 36 x 4 slot of win.
// *used = false (nothing enqueued) when the graph keeps no static triangles,
// has fewer than 2^20 non-self-loop edges (unless TM_TRI_STATIC=1; =0 turns
// the path off), or the calling thread has switched the path off; then the
// incidence-list sweep must count them.  Allocates per-thread workspace and reads two sizes
// back to the host (the stream is synchronised).  shared: other kernels of
// the pass run beside it on other streams (it then takes a smaller grid).
tm_status tm_tri_static_weight(const tm_graph *g, int64_t delta, int64_t s, int64_t L, uint64_t seed, double p,
                               const int32_t *kidx, const uint64_t *wfx, uint64_t *out, uint64_t *win,
                               hipStream_t st, uint64_t pass, bool shared, bool *used);
// On or off for the calling thread (the query server decides per batch).
void tm_tri_static_enable(bool on);
// A grant hook for the calling thread (nullptr: none).  With one, each call
// asks it, before each of its allocation steps, for the device bytes its
// workspace needs in all so far; a refusal leaves the call's triangles to the
// incidence lists.  The static triangles are then not built by the call
// (tm_tri_static_prepare builds them).
typedef bool (*tm_st_grant_fn)(void *ctx, int64_t bytes);
void tm_tri_static_set_grant(tm_st_grant_fn fn, void *ctx);
// Builds the static triangles of a graph that takes the path by default
// (2^20 edges or more); *kept: they are kept and estimates will use them.
tm_status tm_tri_static_prepare(tm_graph *g, hipStream_t st, bool *kept);
bool tm_tri_static_kept(const tm_graph *g);
// Work counts of that path (tm_tri_static_census); TM_EUNSUPPORTED when the
// graph keeps no static triangles.
tm_status tm_tri_static_census_impl(const tm_graph *g, int64_t delta, int64_t s, int64_t L, uint64_t seed, double p,
                                    tm_tri_census *c, hipStream_t st);

// Largest delta for the sweep counter's histogram mode (36 histograms).
#define TM_MAX_SWEEP_HIST_DELTA ((int64_t)1 << 20)

// ------------------------------------------------------------ profiling

// Opt-in kernel timing with HIP events recorded on the launch stream.
// tm_prof_begin returns a token (nullptr when profiling is off) that
// tm_prof_end closes; tm_prof_collect resolves finished events into the
// per-kernel totals (call after the stream has been synchronised).  Kernels
// that run concurrently as one pass share a nonzero pass id (tm_prof_pass);
// the longest of them, the one the pass waits for, is also credited under
// "crit:<name>".
uint64_t tm_prof_pass();
// true while timing runs in serial mode (tm_profile_enable(2)): the kernels
// of a pass then run one after another on the caller's stream, so that each
// one's duration is its own
bool tm_prof_serial();
void *tm_prof_begin(const char *name, hipStream_t st, uint64_t pass = 0);
void tm_prof_end(void *token, hipStream_t st);
void tm_prof_collect();

// ------------------------------------------------------------ batching

// Batched estimates of one three-edge motif (sweep code) for n_seeds seeds in
// one persistent, hipGraph-captured launch (see tm_batch.hip).
tm_status tm_batch_run(const tm_graph *g, int32_t code, int64_t delta, int64_t L, double p, int64_t n_seeds,
                       const uint64_t *seeds, int64_t tile, int64_t bpc, double *est, tm_u128 *kept,
                       hipStream_t st);
// Autotuned (tile, work-groups per CU) for the batched estimator.
tm_status tm_batch_tune(const tm_graph *g, int32_t code, int64_t delta, int64_t L, double p, int64_t *tile,
                        int64_t *bpc, hipStream_t st);
void tm_batch_forget(const tm_graph *g);
void tm_batch_release_plans(const tm_graph *g);
// Estimates of n three-edge-motif queries (sweep codes, each with its own
// delta, window length L, p and seed) in one launch sequence, captured in a
// hipGraph and replayed (capture) or enqueued on st as it is, and the device
// bytes that takes.
tm_status tm_batch_mixed(const tm_graph *g, int64_t n, const int32_t *code, const int64_t *delta, const int64_t *L,
                         const double *p, const uint64_t *seeds, double *est, tm_u128 *kept, hipStream_t st,
                         bool capture = true);
// tm_estimate_mixed with the same choice (the query server enqueues)
tm_status tm_estimate_mixed_ex(const tm_graph *g, int32_t n, const tm_est_query *q, double *estimates,
                               tm_u128 *kept_counts, hipStream_t st, bool capture);
int64_t tm_batch_mixed_bytes(const tm_graph *g, int64_t n, const int64_t *delta, const int64_t *L);

// ------------------------------------------------------------ 4-edge stars

// Whether M is a four-edge star whose first two edges join the center to
// the same leaf, (x,a),(x,a),(x,b),(x,c) with a, b, c distinct; d[k] is the
// direction of edge k at the center (0: it leaves the center, 1: it enters).
bool tm_star4_shape(const tm_motif *M, uint32_t d[4]);
// Its counts (mode 0), counts and 52-bit fixed-point weighted sums (mode 1,
// window length L), or counts and the duration histogram (mode 2, hist_dev:
// delta + 1 bins {lo, hi}, zeroed here); windowed 0: all anchors, 1: anchors
// in windows kept by (s, L, seed, p), 2: every edge in [s, L].  out: count
// lo/hi, weight lo/hi.
tm_status tm_star4_run(const tm_graph *g, const tm_motif *M, int mode, int64_t delta, int windowed, int64_t s, int64_t L,
                       uint64_t seed, double p, uint64_t out[4], uint64_t *hist_dev, hipStream_t st);
// Device bytes of one query (workspace; the first query on a graph also
// builds its ranks: tm_star4_build_bytes).
int64_t tm_star4_bytes(const tm_graph *g, int64_t delta);
int64_t tm_star4_build_bytes(const tm_graph *g);
