/*
 * tm.h -- C ABI of the MI355X (gfx950) temporal-motif library.
 *
 * What it computes (Liu, Benson, Charikar, "A sampling framework for counting
 * temporal motifs", WSDM'19):
 *
 *  - the exact number C_M of delta-instances of a temporal motif M
 *    (Sec. 2, Definitions "temporal motif" and "motif delta-instance"):
 *    time-ordered sequences of distinct temporal edges, with strictly
 *    increasing times (Definition "motif duration"), that map onto M's edges
 *    in order through a bijection of nodes, and whose first and last times
 *    differ by at most delta (inclusive);
 *
 *  - the unbiased estimate Z of Algorithm 1 (Sec. 4) with one shift (b = 1)
 *    and the same sampling probability q_j = p for every window: times are
 *    normalised to start at 0, the shift s is drawn uniformly from
 *    {-c delta + 1, ..., 0}, window j covers [s + (j-1) c delta,
 *    s + j c delta - 1], each window is kept when its uniform draw is below
 *    p, each kept window is counted exactly, and an instance of duration
 *    Delta adds 1 / ((1 - Delta / (c delta)) p)  (equation "estimator").
 *
 * Conventions shared by every entry point:
 *
 *  - Every function returns a tm_status.  Outputs are written only on TM_OK;
 *    no exception or signal crosses the ABI.
 *  - hip_stream is a hipStream_t passed as void* (NULL = the default
 *    stream).  Each call enqueues its device work on that stream and returns
 *    after it has completed; results are host values.
 *  - A tm_graph is immutable once loaded; calls that only read it may run
 *    concurrently from different host threads on different streams.
 *  - Motifs use node labels 0..k-1 in order of first appearance (edge 0 is
 *    (0,1)); no self-loops; every edge after the first touches a node of an
 *    earlier edge (prefix-connected); 1 <= l <= 4 edges.  Other motifs give
 *    TM_EUNSUPPORTED (l > 4, not prefix-connected) or TM_EINVAL.
 *  - Graph self-loop edges are accepted and never match (the node map of an
 *    instance is a bijection).  Tied timestamps are accepted; tied edges
 *    never share an instance.
 */
#ifndef TM_H
#define TM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TM_OK = 0,
    TM_EINVAL = 1,        /* bad argument (sizes, ids, delta, c, p, motif form) */
    TM_EUNSUPPORTED = 2,  /* motif outside the supported class                */
    TM_ENOMEM = 3,        /* device or host allocation failed                 */
    TM_EBUDGET = 4,       /* request exceeds the caller's memory budget       */
    TM_EOVERFLOW = 5,     /* result does not fit the requested width          */
    TM_EDEVICE = 6        /* a HIP runtime call failed                        */
} tm_status;

/* exact non-negative 128-bit count: value = hi * 2^64 + lo */
typedef struct { uint64_t lo, hi; } tm_u128;

/* motif edges (src[i] -> dst[i]), i = 0..l-1, in the motif's time order */
typedef struct { int32_t l; int32_t src[4]; int32_t dst[4]; } tm_motif;

typedef struct tm_graph tm_graph;

typedef struct {
    int64_t m;            /* temporal edges                                  */
    int64_t n;            /* nodes                                           */
    int64_t t_min;        /* smallest input time (normalisation origin)      */
    int64_t t_span;       /* largest normalised time t - t_min               */
    int64_t n_pairs;      /* distinct directed (u, v) pairs, u != v          */
    int64_t device_bytes; /* device memory held by the graph                 */
    int64_t exact_table_bytes; /* of which the exact-count tables (0: none)  */
} tm_graph_info;

/* Optional diagnostics of one estimate.  Pointers are caller-owned host
   buffers (each may be NULL); the first `cap` kept windows are written. */
typedef struct {
    int64_t shift;        /* s, in {-c delta + 1, ..., 0}                    */
    int64_t n_windows;    /* J = 1 + ceil(t_span / (c delta))                */
    int64_t n_kept;       /* windows kept by the Bernoulli draws             */
    tm_u128 kept_count;   /* exact instance count summed over kept windows   */
    int64_t cap;          /* capacity of kept_ids / win_counts               */
    int64_t *kept_ids;    /* kept window indices j (1-based), ascending      */
    uint64_t *win_counts; /* exact count of each kept window (low 64 bits)   */
    uint64_t *hist_lo;    /* delta+1 bins: N(Delta) summed over kept windows */
    uint64_t *hist_hi;    /*   (high 64 bits of each bin)                    */
} tm_est_info;

/*
 * Load a temporal graph (Sec. 2: tuples (u_i, v_i, t_i), i = 1..m) onto the
 * current device.  src/dst are int32 node ids in [0, n_nodes), t int64
 * times; the three arrays have m entries and live in host memory
 * (on_device = 0) or device memory (on_device = 1).  They are copied; the
 * library keeps no caller pointer.  The graph is stored time-sorted with
 * per-node time-sorted incidence lists (device radix sort + CSR build).
 * The device memory that loads and exact triangle counts free (their
 * temporaries) is kept, up to 2 GiB per host thread, for the next such call
 * on the same thread; it goes back to the device when one of their
 * allocations runs out of memory or the thread ends.
 * Errors: TM_EINVAL (m < 0, n_nodes <= 0, an id outside [0, n_nodes), NULL
 * array with m > 0), TM_ENOMEM, TM_EDEVICE.  *out is owned by the caller
 * until tm_free_graph.
 */
tm_status tm_load_graph(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t m,
                        int32_t n_nodes, int32_t on_device, void *hip_stream, tm_graph **out);

/* Flags of tm_load_graph_ex. */
enum {
    TM_LOAD_ON_DEVICE = 1,       /* src/dst/t are device pointers                     */
    TM_LOAD_NO_EXACT_TABLES = 2  /* skip the exact-count tables (see below)           */
};

/*
 * tm_load_graph with flags.  Unless TM_LOAD_NO_EXACT_TABLES is set, the load
 * also builds the exact-count tables (192 B per edge: per pair entry and
 * endpoint, prefix sums of the counts the exact 2-node and star motif counts
 * are range sums of), when they fit in a quarter of the free device memory;
 * without them exact counts scan every anchor's window instead.  Results are
 * identical either way.  Other arguments and errors as tm_load_graph.
 */
tm_status tm_load_graph_ex(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t m,
                           int32_t n_nodes, uint32_t flags, void *hip_stream, tm_graph **out);

/* Release a graph and its device memory.  NULL is ignored. */
void tm_free_graph(tm_graph *g);

/* Sizes of a loaded graph. */
tm_status tm_graph_info_get(const tm_graph *g, tm_graph_info *info);

/*
 * Exact count C_M of delta-instances of M in the whole graph (Sec. 2,
 * Definition "motif delta-instance").  delta >= 0.  Exact 128-bit result.
 */
tm_status tm_count_exact(const tm_graph *g, const tm_motif *M, int64_t delta, tm_u128 *count,
                         void *hip_stream);

/* As tm_count_exact; TM_EOVERFLOW when the count is 2^63 or more. */
tm_status tm_count_exact_i64(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t *count,
                             void *hip_stream);

/*
 * Exact counts and duration histograms of n_motifs motifs in one pass.
 * counts[i] receives C_M of motifs[i].  hist_lo/hist_hi (nullable, host,
 * n_motifs * (delta + 1) entries, motif-major) receive the number of
 * instances of each duration Delta = t_l - t_1 (Definition "motif
 * duration"); with histograms delta must be <= 2^26 (else TM_EUNSUPPORTED).  The pass shares the graph scans between motifs when all of
 * them have three edges.
 */
tm_status tm_count_exact_multi(const tm_graph *g, int32_t n_motifs, const tm_motif *motifs,
                               int64_t delta, tm_u128 *counts, uint64_t *hist_lo,
                               uint64_t *hist_hi, void *hip_stream);

/*
 * Exact counts inside one time window: the counting subroutine A(T', M,
 * delta) of Sec. 4 applied to the sub-graph T' of edges with input time in
 * [t_lo, t_hi] (the per-window step of Algorithm 1).  counts[i] for
 * motifs[i]; all three-edge motifs share one pass.
 */
tm_status tm_count_window(const tm_graph *g, int32_t n_motifs, const tm_motif *motifs, int64_t delta,
                          int64_t t_lo, int64_t t_hi, tm_u128 *counts, void *hip_stream);

/*
 * Per-anchor counts: for each listed edge (index into the caller's input
 * arrays as given to tm_load_graph), the number of delta-instances whose
 * first edge is that edge and whose edges all have normalised time
 * <= win_end[i] (win_end NULL: no window).  out[i] is 64-bit (TM_EOVERFLOW
 * when one does not fit).  Host arrays of n_anchor entries.
 */
tm_status tm_count_anchors(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t n_anchor,
                           const int64_t *anchor, const int64_t *win_end, uint64_t *out,
                           void *hip_stream);

/*
 * The estimate Z of Algorithm 1 (Sec. 4) for one shift with q_j = p.
 * delta >= 1, c >= 2 (at c = 1 an instance of duration delta would have
 * containment probability 0), 0 < p <= 1, any seed.  TM_EINVAL when c delta
 * exceeds 2^61 or the graph's time span exceeds 2^63 - 1 - 2 c delta;
 * TM_EUNSUPPORTED when delta > 2^26 (the histogram has delta + 1 bins).  The random numbers come
 * from Philox4x32-10 keyed by the seed: the shift is -(X mod c delta) for the
 * draw X at counter (0, 0, 0, 0); window j is kept when (Y_j >> 11) 2^-53 < p
 * for the draw Y_j at counter (j mod 2^32, j div 2^32, 0, 1); a draw is the
 * 64-bit (word1 << 32) | word0.  Kept windows are counted exactly; the
 * duration histogram N(Delta) summed over kept windows is weighted in FP64
 * in ascending Delta with compensated summation:
 * Z = (1/p) sum_Delta N(Delta) c delta / (c delta - Delta).
 * info (nullable) receives the diagnostics above.
 */
tm_status tm_estimate(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t c, double p,
                      uint64_t seed, double *estimate, tm_est_info *info, void *hip_stream);

/*
 * Estimates for n_motifs motifs under one (delta, c, p, seed): the same
 * shift and kept windows for all of them (one pass when all have three
 * edges).  estimates[i] for motifs[i]; kept_counts (nullable) the exact
 * per-motif instance counts over the kept windows.
 *
 * Three-node triangle motifs (their three edges on three node pairs) are
 * summed over the graph's static triangles on graphs of at least 2^20
 * non-self-loop edges (tm_tri_static_census describes that work; the static
 * triangles are found on the first such call and kept with the graph), over
 * the incidence lists otherwise; both give the same bits.  The environment
 * variable TM_TRI_STATIC=0 keeps the incidence lists, =1 takes the static
 * triangles on any graph.  The query server's slot threads take them for a
 * lone triangle estimate charged their workspace, within that charge (else
 * the incidence lists).  The same holds for tm_estimate and tm_estimate_q.
 */
tm_status tm_estimate_multi(const tm_graph *g, int32_t n_motifs, const tm_motif *motifs,
                            int64_t delta, int64_t c, double p, uint64_t seed, double *estimates,
                            tm_u128 *kept_counts, void *hip_stream);

/*
 * Algorithm 1 of Sec. 4 with b shifts and the window probabilities the paper
 * uses (equation heuristic_q): window j of shift k is kept with probability
 * q_j = min(1, r |T_j| / |T|), where |T_j| counts the edges (self-loops
 * included) whose normalised time lies in I_j and |T| = m; a q_j above 1 is
 * clamped, which keeps the estimate unbiased.  A kept window adds
 * Y_{s,j} / q_j, Y_{s,j} being its weighted count w(I_j) (the sum over its
 * instances of 1 / (1 - Delta / (c delta))), and the estimate is the mean
 * over the b shifts.  Shift k takes its shift from draw (0, k, domain 0)
 * and its window uniforms from draws (j, k, domain 1) of the seed's
 * Philox4x32-10 stream, so shift 0 is tm_estimate's shift.
 * Motifs: up to four edges, prefix-connected (TM_EUNSUPPORTED otherwise),
 * n_motifs >= 1.  When every motif has three edges, one windowed sweep per
 * shift gives each kept window's exact fixed-point Y_{s,j}; otherwise each
 * kept window and motif is counted by the generic counter with its duration
 * histogram, weighted in FP64 in ascending Delta (delta up to 2^26).
 * delta >= 1, c >= 2, r > 0 and finite, b >= 1.  estimates: host array of
 * n_motifs.  info (nullable, host memory, caller-owned): n_kept (out) = the
 * kept windows over all shifts; with cap > 0 the first cap of them, in order
 * of (k, j), are described in win_k[cap], win_j[cap] (1-based), win_q[cap]
 * and win_y[cap * n_motifs] (one row per window: Y_{s,j} of each motif).
 * Errors: TM_EINVAL (bad arguments, or null info arrays with cap > 0),
 * TM_EUNSUPPORTED (a motif over four edges or not prefix-connected, more
 * than 2^30 windows, delta above 2^26 with a motif of other than three edges),
 * TM_ENOMEM, TM_EDEVICE.  Outputs are written only on TM_OK.
 */
/*
 * Algorithm 1 (Sec. 4, one shift, q_j = p) with the windows visited in time
 * order and only one kept window's edges on the device at a time: the
 * streaming, memory-bounded use the paper describes after choosing the
 * sampling probabilities.  The edges are host arrays (src, dst, t, m; node
 * ids below n_nodes; device arrays: TM_EINVAL) sorted by non-decreasing
 * time; the library checks the
 * order on the device in bounded chunks (TM_EINVAL when unsorted) and
 * validates the ids of every window it reads.  Per kept window it uploads
 * that window's edges, builds a graph of them and sweeps it, so the device
 * holds one window at a time.  Each motif's result is tm_estimate's on the
 * whole graph with the same seed, to the last bit: three-edge motifs sum the
 * same exact fixed-point integers over the window sweeps; other motifs (up
 * to four edges, prefix-connected; delta up to 2^26) add the windows'
 * integer duration histograms on the device and weight the total once, as
 * tm_estimate does.  Kept counts are exact.  estimates[n_motifs], kept_counts[n_motifs]
 * (nullable): host.  info (nullable, host): the shift, J, the kept windows,
 * the edges of the largest kept window (what is resident at once) and the
 * device bytes of its graph.  Errors as tm_estimate_multi and tm_load_graph.
 */
typedef struct {
    int64_t shift;
    int64_t n_windows;
    int64_t n_kept;
    int64_t max_window_edges;
    int64_t peak_graph_bytes;
} tm_stream_info;
tm_status tm_estimate_stream(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t m, int32_t n_nodes,
                             int32_t n_motifs, const tm_motif *motifs, int64_t delta, int64_t c, double p,
                             uint64_t seed, double *estimates, tm_u128 *kept_counts, tm_stream_info *info,
                             void *hip_stream);

typedef struct {
    int64_t n_kept;
    int64_t cap;
    int64_t *win_k;
    int64_t *win_j;
    double *win_q;
    double *win_y;
} tm_q_info;
tm_status tm_estimate_q(const tm_graph *g, int32_t n_motifs, const tm_motif *motifs, int64_t delta, int64_t c,
                        double r, int32_t b, uint64_t seed, double *estimates, tm_q_info *info, void *hip_stream);

/*
 * Batched estimator: n_seeds independent estimates of one motif (each seed
 * draws its own shift and window samples, Algorithm 1's loop over shifts run
 * as separate estimators); estimates[k] equals tm_estimate with seeds[k].
 * For the 36 three-edge motifs all kept windows of all seeds are counted in
 * one persistent launch: node-aligned tiles of at most `tile` anchors are
 * queued per (seed, tile) that meets a kept window, and resident
 * wavefronts take tasks from the shared queue (work stealing).  The kernel
 * sequence is captured once as a hipGraph per (graph, motif, delta, c, p,
 * n_seeds, tile, grid) and replayed with the new seeds.  tile = 0 uses the
 * autotuned tile and grid (tm_batch_config); a nonzero tile runs with 8
 * work-groups per CU.  Other motifs run seed by seed.
 * kept_counts (nullable) receives each seed's exact count over its kept
 * windows.  Plans are cached with the graph and released by tm_free_graph.
 * Calls with the same (motif, delta, c, p, n_seeds, tile) share one plan:
 * concurrent ones (other threads, other streams) run it one after another.
 */
tm_status tm_estimate_batch(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t c,
                            double p, int32_t n_seeds, const uint64_t *seeds, int32_t tile,
                            double *estimates, tm_u128 *kept_counts, void *hip_stream);

/*
 * Estimates of n queries on one graph, each with its own motif, delta, c, p
 * and seed (Algorithm 1 once per query).  The queries with three-edge motifs
 * run together in one persistent, work-stealing launch replayed from a
 * captured hipGraph: node-aligned tiles of 256 anchors are queued per
 * (tile, query) that meets a window the query keeps, one kernel per sweep
 * class (the classes as parallel branches of the graph).  Other motifs (up to
 * four edges) run one after another through the generic counter.
 * estimates[i] and kept_counts[i] (nullable: exact counts over the kept
 * windows) are each query's tm_estimate result, to the last bit.  Host
 * arrays of n entries.  Errors: as tm_estimate for any query.
 */
typedef struct {
    tm_motif motif;
    int64_t delta;
    int64_t c;
    double p;
    uint64_t seed;
} tm_est_query;
tm_status tm_estimate_mixed(const tm_graph *g, int32_t n, const tm_est_query *q, double *estimates,
                            tm_u128 *kept_counts, void *hip_stream);

/*
 * Autotuner of the batched estimator: times candidate tile sizes
 * {64, 256, 1024} and work-groups per CU {8, 16} on 2 seeds and
 * returns (and caches for the graph) the fastest pair.  Three-edge motifs
 * only (TM_EUNSUPPORTED otherwise).
 */
tm_status tm_batch_config(const tm_graph *g, const tm_motif *M, int64_t delta, int64_t c, double p,
                          int32_t *tile, int32_t *blocks_per_cu, void *hip_stream);

/*
 * Releases the batched estimator's cached state of graph g: captured plans
 * and the stored anchor values (32 B per incidence entry per (motif, delta,
 * c)), after waiting for hip_stream.  Tuning results are kept.  The next
 * tm_estimate_batch rebuilds what it needs.  A plan that a concurrent
 * tm_estimate_batch is running stays alive until that run ends.
 */
tm_status tm_batch_release(const tm_graph *g, void *hip_stream);

/*
 * Allocation-free variant of tm_estimate_multi, for callers that cannot
 * allocate device memory: code under hipGraph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The estimates are those of
 * tm_estimate_multi for the same arguments, to the last bit (the same
 * kernels and the same exact fixed-point sums).
 *
 *  - Motifs: the 36 three-edge motifs on two or three nodes only
 *    (TM_EUNSUPPORTED otherwise); n_motifs >= 1.  delta <= TM_NOALLOC_MAX_DELTA
 *    (TM_EUNSUPPORTED above it); other argument errors as tm_estimate.
 *  - Outputs are caller-owned DEVICE arrays: estimates_dev[n_motifs]
 *    (double) and kept_dev[n_motifs] (nullable; exact kept-window counts).
 *  - Work space: a library-owned static device array of
 *    8 (168 + TM_NOALLOC_MAX_DELTA + 1) bytes (about 8 MiB) per GPU, held
 *    until the process ends; no hipMalloc, hipFree or other allocation is
 *    made.  Every call on one GPU shares that array: calls that overlap on one
 *    GPU (different streams or host threads without ordering) race and give
 *    wrong results.  Each call clears what it reads.
 *  - The pass runs its kernels one after another on hip_stream and the call
 *    returns once they are enqueued, without waiting: results are valid when
 *    the stream reaches that point (synchronize it, or capture the call).
 *    Errors of kernels that have not run yet surface in later HIP calls.
 */
#define TM_NOALLOC_MAX_DELTA ((int64_t)1048575)
tm_status tm_estimate_multi_noalloc(const tm_graph *g, int32_t n_motifs, const tm_motif *motifs, int64_t delta,
                                    int64_t c, double p, uint64_t seed, double *estimates_dev,
                                    tm_u128 *kept_dev, void *hip_stream);

/* ------------------------------------------------------------------ serving */

typedef struct tm_server tm_server;

typedef struct {
    int32_t graph;     /* id from tm_server_add_graph                         */
    int32_t kind;      /* 0: exact count (tm_count_exact); 1: estimate         */
    tm_motif motif;
    int64_t delta;
    int64_t c;         /* estimate only                                       */
    double p;          /* estimate only                                       */
    uint64_t seed;     /* estimate only                                       */
} tm_query;

typedef struct {
    tm_status status;    /* TM_EBUDGET when the query alone exceeds the budget */
    tm_u128 count;       /* exact count; for estimates the kept-window count   */
    double estimate;     /* kind 1                                            */
    double latency_ms;   /* submit to result                                  */
    double queue_ms;     /* submit to start on a slot                         */
    int32_t batch_size;  /* queries answered by the same device pass          */
    int32_t slot;
    int64_t ws_charged;  /* device bytes the batch was charged against the budget */
    int64_t ws_measured; /* device bytes the batch held at its peak (measured)  */
} tm_result;

typedef struct {
    int64_t submitted, completed, rejected, batches;
    double p50_ms, p99_ms, mean_ms;   /* nearest-rank latency percentiles   */
    double wall_s;                    /* first submit to last completion     */
    double edges_per_s;               /* graph edges of completed queries / wall_s */
    int64_t budget_bytes, peak_bytes; /* admitted workspace, high-water mark */
    int64_t measured_max_bytes;       /* largest measured batch workspace    */
    int64_t over_charge;              /* batches that held more than charged */
    int64_t uncollected;              /* results ready but not yet waited for */
} tm_server_stats;

/*
 * Query server with continuous batching.  `slots` worker threads, each with
 * its own HIP stream, run batches concurrently; a dispatcher admits the
 * oldest queued query whose device workspace fits what is left of
 * budget_bytes, merges every queued query that can share its device work
 * (exact counts of three-edge motifs on the same graph and delta share one
 * sweep; estimates of three-edge motifs on the same graph share the launch
 * sequence of tm_estimate_mixed, enqueued on the slot's stream rather than
 * captured, whatever their motifs, deltas, c, p and seeds; a lone estimate,
 * or one on a heavy graph, takes tm_estimate_multi's sweep; a lone triangle
 * estimate may sum its triangles over the graph's static triangles, which
 * tm_server_add_graph finds for graphs of 2^20 edges or more: that path's
 * per-call workspace is known only on the device, so the running batch asks
 * for it before allocating and its charge grows by what fits the budget then,
 * or the estimate counts its triangles over the incidence lists), up to 256
 * per batch, and starts it on a
 * free slot; batches on graphs with at least an eighth of the largest
 * graph's edges take at most half the slots while lighter graphs are
 * resident.  A batch is charged the
 * device bytes its path allocates, and the bytes it really allocated are
 * measured and reported beside the charge (tm_result, tm_server_stats); the
 * grow-only workspaces a slot thread keeps between batches are measured
 * after each batch and counted against the budget too (an idle slot frees
 * them when the oldest query would not fit otherwise), so budget_bytes
 * bounds the device memory the server's threads hold beyond the graphs.
 * Queries that arrive while others run are admitted as slots and memory
 * free up.  A result is the same whether its
 * query ran alone or in a batch.  Graphs must stay loaded while the server
 * uses them.  tm_server_wait blocks until the ticket's result is ready
 * (TM_EINVAL for an unknown or already collected ticket; a collected result
 * is dropped from the server, one byte per ticket stays); tm_server_destroy
 * completes queued queries with TM_EDEVICE and joins the threads.
 */
tm_status tm_server_create(int32_t slots, int64_t budget_bytes, tm_server **out);
tm_status tm_server_add_graph(tm_server *s, const tm_graph *g, int32_t *graph_id);
tm_status tm_server_submit(tm_server *s, const tm_query *q, int64_t *ticket);
tm_status tm_server_wait(tm_server *s, int64_t ticket, tm_result *result);
tm_status tm_server_stats_get(tm_server *s, tm_server_stats *stats);
void tm_server_destroy(tm_server *s);

/*
 * Kernel timing (off by default).  When enabled, the library brackets its
 * main kernel launches with HIP events on the stream each kernel runs on and
 * adds the elapsed times per kernel name ("sweep3_{fwd,bwd,tri}_count",
 * "sweep3_{fwd,bwd,tri}_weight", "sweep3_{fwd,bwd,tri}_hist",
 * "count_generic", "count_batch", "count_batch_stored",
 * "batch_anchor_values").  The sweep kernels of one pass run concurrently;
 * the longest of them, which the pass waits for, is also credited under
 * "crit:<name>" (one launch per pass).  tm_profile_read returns the total
 * milliseconds and the number of launches so far (zeros for a name never
 * timed).  on = 2 also runs the kernels of each pass one after another on
 * the caller's stream (a diagnostic: each duration is then the kernel's own,
 * and a pass takes longer); on = 1 times without changing how kernels run,
 * 0 stops timing.  Other values: TM_EINVAL.
 */
tm_status tm_profile_enable(int32_t on);
tm_status tm_profile_reset(void);
tm_status tm_profile_read(const char *kernel, double *total_ms, int64_t *launches);

/*
 * Work census of the three-edge sweeps, used to express kernel time as
 * algorithmic bytes per second.  tm_sweep_census covers the exact sweeps at
 * span delta over the whole graph:
 *   anchors       incidence entries (two per non-self-loop edge)
 *   fwd_entries   list entries the forward sweeps scan (later entries of
 *                 the anchor's list within delta)
 *   bwd_entries   list entries the backward sweep scans (earlier ones)
 *   tri_anchors   entries of the ranked sublists (those whose other endpoint
 *                 ranks above the list's owner, rank = (list length, node
 *                 id)): the exact triangle sweep's anchors
 *   tri_entries   ranked-sublist entries that sweep scans
 *   tri_lookups   scanned entries that lead to another node than the
 *                 anchor's (one closing-pair lookup each)
 *   tri_pairs     of those, the ones whose node differs from the previous
 *                 lookup's (the pair's id and metadata are read)
 * tm_sweep_census_est covers the estimate's weighted sweeps for (delta, c,
 * p, seed): the same fields restricted to anchors in kept windows and to
 * entries inside the anchor's window; there the triangle sweep runs over
 * the full lists, so tri_anchors = anchors and tri_entries = fwd_entries.
 *   tri_probes    binary-search probes of a plain lookup of the closing
 *                 pair's middle count, ceil(log2(n + 1)) per search of a pair
 *                 timeline of n entries: the exact sweep searches at t_j and
 *                 t_j - delta per lookup and, per change of pair, probes once
 *                 to find it and searches at t_i and at the window end; the
 *                 weighted sweep searches at t_j per lookup and, per change,
 *                 probes once and searches at t_i
 * Ties with the anchor's time are left out of tri_lookups and tri_pairs, as
 * the sweeps leave them out.  Within a list, entries tied in time follow the
 * input order of their edges (an edge's source entry before its destination
 * entry), which tri_pairs depends on.
 */
typedef struct {
    int64_t anchors, fwd_entries, bwd_entries;
    int64_t tri_anchors, tri_entries, tri_lookups, tri_pairs;
    int64_t tri_probes;
} tm_census;

tm_status tm_sweep_census(const tm_graph *g, int64_t delta, tm_census *out, void *hip_stream);
tm_status tm_sweep_census_est(const tm_graph *g, int64_t delta, int64_t c, double p, uint64_t seed,
                              tm_census *out, void *hip_stream);

/*
 * Work census of the weighted triangle sums of an estimate for (delta, c,
 * p, seed) as tm_estimate_multi computes them for triangle motifs: over the
 * static triangles {u0, u1, u2} (three node pairs joined by edges; Sec. 2,
 * the three edges of a triangle instance lie on the three pairs), inside
 * each kept window (Sec. 4, Algorithm 1).
 *   triangles  static triangles of the graph
 *   units      (static triangle, kept window) with edges on all three pairs
 *              inside the window
 *   tasks      work items: per unit, six roles (the pair of the middle edge,
 *              and which other pair holds the first edge), each cut into
 *              chunks of 32 entries of the lighter of the first- and
 *              last-edge pairs (the driver)
 *   drivers    driver entries whose window range holds a middle edge and a
 *              candidate edge on the third pair
 *   steps      64-entry steps over those candidates
 *   combos     (first, last) edge pairs visited (candidates in the steps)
 * TM_EUNSUPPORTED when the graph keeps no static triangles (too many
 * candidates to enumerate, or a pair with 2^28 edges or more); estimates
 * then count triangles over the incidence lists.  Synchronises the stream.
 */
typedef struct {
    int64_t triangles, units, tasks, drivers, steps, combos;
} tm_tri_census;

tm_status tm_tri_static_census(const tm_graph *g, int64_t delta, int64_t c, double p, uint64_t seed,
                               tm_tri_census *out, void *hip_stream);

/* Human-readable name of a status code (static storage). */
const char *tm_strerror(tm_status s);

/* Library version string (static storage). */
const char *tm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TM_H */
