/*
 * CPU oracle for delta-temporal motif counting and the sampling estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library under
 * paper_1810_00980_amd/ links, loads or calls this file; only tests/,
 * __graft_entry__.smoke() and the CPU-baseline leg of bench.py use it.  It
 * shares no code, header, table or helper with the HIP path.
 *
 * Everything here is deliberately plain and slow:
 *
 *  - orc_count: brute force over time-ordered edge sequences (paper Sec. 2,
 *    Definitions "temporal motif", "motif delta-instance" and "motif
 *    duration").  Edges are put in (time, input index) order; for every anchor
 *    edge, later edges are tried one motif edge at a time, binding the motif's
 *    nodes to graph nodes through an injective map, and a completed sequence
 *    adds one to the histogram bin of its duration t_l - t_1.  Times inside an
 *    instance must increase strictly (the duration definition writes
 *    t_1 < t_2 < ... < t_l), the span bound t_l - t_1 <= delta is inclusive,
 *    and with a window [win_lo, win_hi] every edge must lie in it (the
 *    sub-graph T_j of Algorithm 1).
 *
 *  - orc_estimate: Algorithm 1 (Sec. 4) with uniform sampling probability
 *    q_j = p and one shift: normalise times to start at 0, J = 1 +
 *    ceil(t_max / (c delta)), draw the shift s uniformly from
 *    {-c delta + 1, ..., 0}, keep window j when its uniform draw is below p,
 *    count each kept window exactly, and add count / ((1 - Delta/(c delta)) p).
 *    Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *    "Parallel random numbers: as easy as 1, 2, 3", SC'11), written here from
 *    that definition.
 *
 *  - orc_weight: the weighting step of Algorithm 1 on an integer duration
 *    histogram, summed in ascending duration order with Neumaier's
 *    compensated summation in IEEE double, then divided by p.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef unsigned __int128 u128;

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 3
#define ORC_EOVERFLOW 5

#define ORC_MAXK 64 /* motif nodes */
#define ORC_MAXL 64 /* motif edges */

/* ------------------------------------------------------------------ order */

/* merge sort of edge indices by (t, index): a total order that keeps ties in
   input order (any order of tied edges gives the same counts, because tied
   edges never share an instance). */
static void msort(int64_t *a, int64_t *tmp, int64_t n, const int64_t *t) {
    if (n < 2) return;
    int64_t h = n / 2;
    msort(a, tmp, h, t);
    msort(a + h, tmp, n - h, t);
    int64_t i = 0, j = h, k = 0;
    while (i < h && j < n) {
        int64_t x = a[i], y = a[j];
        if (t[y] < t[x] || (t[y] == t[x] && y < x)) tmp[k++] = a[j++];
        else tmp[k++] = a[i++];
    }
    while (i < h) tmp[k++] = a[i++];
    while (j < n) tmp[k++] = a[j++];
    memcpy(a, tmp, (size_t)n * sizeof(int64_t));
}

static int64_t *time_order(int64_t m, const int64_t *t) {
    int64_t *ord = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
    int64_t *tmp = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
    if (!ord || !tmp) { free(ord); free(tmp); return NULL; }
    for (int64_t i = 0; i < m; ++i) ord[i] = i;
    msort(ord, tmp, m, t);
    free(tmp);
    return ord;
}

/* --------------------------------------------------------------- matching */

typedef struct {
    const int32_t *src, *dst;
    const int64_t *t;
    const int64_t *ord;
    int64_t m;
    int l, k;
    const int32_t *ms, *md;
    int64_t delta, win_hi;
    int64_t f[ORC_MAXK];   /* motif node -> graph node, -1 when unbound */
    int64_t t_first;
    u128 total;
    uint64_t *hist;        /* delta + 1 bins or NULL */
    int overflow;
} ctx_t;

static int64_t sat_add(int64_t a, int64_t b) {
    /* b >= 0 here */
    if (a > INT64_MAX - b) return INT64_MAX;
    return a + b;
}

/* try to bind motif node x to graph node g; returns 1 when consistent.
   *newly is set when the binding was created here (to undo it later). */
static int bind(ctx_t *c, int x, int64_t g, int *newly) {
    *newly = 0;
    if (c->f[x] >= 0) return c->f[x] == g;
    for (int y = 0; y < c->k; ++y)
        if (c->f[y] == g) return 0; /* injective */
    c->f[x] = g;
    *newly = 1;
    return 1;
}

static void extend(ctx_t *c, int level, int64_t pos, int64_t t_prev, int64_t tlim) {
    if (level == c->l) {
        int64_t d = t_prev - c->t_first;
        c->total += 1;
        if (c->hist) {
            if (c->hist[d] == UINT64_MAX) c->overflow = 1;
            c->hist[d] += 1;
        }
        return;
    }
    int u = c->ms[level], v = c->md[level];
    for (int64_t q = pos + 1; q < c->m; ++q) {
        int64_t e = c->ord[q];
        int64_t te = c->t[e];
        if (te > tlim) break;
        if (te == t_prev) continue; /* strictly increasing times */
        int nu, nv;
        if (!bind(c, u, c->src[e], &nu)) continue;
        if (!bind(c, v, c->dst[e], &nv)) { if (nu) c->f[u] = -1; continue; }
        extend(c, level + 1, q, te, tlim);
        if (nv) c->f[v] = -1;
        if (nu) c->f[u] = -1;
    }
}

static int motif_ok(int l, const int32_t *ms, const int32_t *md, int *k_out) {
    if (l < 1 || l > ORC_MAXL) return 0;
    int k = 0;
    for (int i = 0; i < l; ++i) {
        if (ms[i] < 0 || md[i] < 0 || ms[i] >= ORC_MAXK || md[i] >= ORC_MAXK) return 0;
        if (ms[i] == md[i]) return 0;
        if (ms[i] + 1 > k) k = ms[i] + 1;
        if (md[i] + 1 > k) k = md[i] + 1;
    }
    *k_out = k;
    return 1;
}

static void anchor_count(ctx_t *c, int64_t q) {
    int64_t e = c->ord[q];
    int64_t te = c->t[e];
    int nu, nv;
    if (te > c->win_hi) return; /* every edge of an instance, the first one too, lies in the window */
    for (int x = 0; x < c->k; ++x) c->f[x] = -1;
    if (!bind(c, c->ms[0], c->src[e], &nu)) return;
    if (!bind(c, c->md[0], c->dst[e], &nv)) return;
    c->t_first = te;
    int64_t tlim = sat_add(te, c->delta);
    if (tlim > c->win_hi) tlim = c->win_hi;
    extend(c, 1, q, te, tlim);
}

/*
 * Count delta-instances of the motif (ms[i] -> md[i], i = 0..l-1, motif nodes
 * labelled 0..k-1) among edges whose times all lie in [win_lo, win_hi].
 * hist (nullable) receives delta+1 bins indexed by duration and is added to,
 * not cleared.  total_lo/hi receive the 128-bit total.
 */
int orc_count(int64_t m, const int32_t *src, const int32_t *dst, const int64_t *t,
              int l, const int32_t *ms, const int32_t *md, int64_t delta,
              int64_t win_lo, int64_t win_hi, uint64_t *hist,
              uint64_t *total_lo, uint64_t *total_hi) {
    int k;
    if (m < 0 || delta < 0 || !motif_ok(l, ms, md, &k)) return ORC_EINVAL;
    int64_t *ord = time_order(m, t);
    if (!ord) return ORC_ENOMEM;
    ctx_t c;
    memset(&c, 0, sizeof c);
    c.src = src; c.dst = dst; c.t = t; c.ord = ord; c.m = m;
    c.l = l; c.k = k; c.ms = ms; c.md = md; c.delta = delta; c.win_hi = win_hi;
    c.hist = hist;
    for (int64_t q = 0; q < m; ++q) {
        int64_t te = t[ord[q]];
        if (te < win_lo || te > win_hi) continue;
        anchor_count(&c, q);
    }
    free(ord);
    *total_lo = (uint64_t)c.total;
    *total_hi = (uint64_t)(c.total >> 64);
    return c.overflow ? ORC_EOVERFLOW : ORC_OK;
}

/*
 * Per-anchor counts: for each listed edge index a (input indexing), the number
 * of instances whose first edge is edge a, with every edge at time
 * <= win_hi[i] (pass INT64_MAX for no window).  out[i] is 64-bit; overflow
 * is reported.  hist (nullable) accumulates the durations of those instances.
 */
int orc_count_anchors(int64_t m, const int32_t *src, const int32_t *dst, const int64_t *t,
                      int l, const int32_t *ms, const int32_t *md, int64_t delta,
                      int64_t n_anchor, const int64_t *anchor, const int64_t *win_hi,
                      uint64_t *out, uint64_t *hist) {
    int k;
    if (m < 0 || delta < 0 || !motif_ok(l, ms, md, &k)) return ORC_EINVAL;
    int64_t *ord = time_order(m, t);
    if (!ord) return ORC_ENOMEM;
    int64_t *pos = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
    if (!pos) { free(ord); return ORC_ENOMEM; }
    for (int64_t q = 0; q < m; ++q) pos[ord[q]] = q;
    ctx_t c;
    memset(&c, 0, sizeof c);
    c.src = src; c.dst = dst; c.t = t; c.ord = ord; c.m = m;
    c.l = l; c.k = k; c.ms = ms; c.md = md; c.delta = delta; c.hist = hist;
    int rc = ORC_OK;
    for (int64_t i = 0; i < n_anchor; ++i) {
        if (anchor[i] < 0 || anchor[i] >= m) { rc = ORC_EINVAL; break; }
        c.total = 0;
        c.win_hi = win_hi ? win_hi[i] : INT64_MAX;
        anchor_count(&c, pos[anchor[i]]);
        if (c.total >> 64) c.overflow = 1;
        out[i] = (uint64_t)c.total;
    }
    free(pos);
    free(ord);
    if (rc != ORC_OK) return rc;
    return c.overflow ? ORC_EOVERFLOW : ORC_OK;
}

/* ----------------------------------------------------------------- Philox */

/* Philox4x32 with 10 rounds.  Each round multiplies counter words 0 and 2 by
   the two round multipliers, mixes the high halves with words 1 and 3 and the
   key, and permutes; the key is bumped by the two Weyl constants between
   rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One 64-bit draw for window index j (domain 1) or the shift (domain 0, j=0)
   of estimator k under key = seed: counter (lo32 j, hi32 j, k, domain);
   the draw is (word1 << 32) | word0. */
uint64_t orc_draw(uint64_t seed, uint64_t j, uint32_t k, uint32_t domain) {
    uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(j >> 32), k, domain};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    return ((uint64_t)o[1] << 32) | (uint64_t)o[0];
}

/* -------------------------------------------------------------- weighting */

static double u128_to_double(uint64_t lo, uint64_t hi) {
    double xh = (double)hi;
    double r = xh * 18446744073709551616.0;
    return r + (double)lo;
}

/* Z = (1/p) * sum_{d=0..delta} N(d) * L / (L - d), ascending d, Neumaier.
   hist_hi may be NULL (all high words zero). Requires L > delta. */
double orc_weight(const uint64_t *hist_lo, const uint64_t *hist_hi, int64_t delta,
                  int64_t L, double p) {
    double sum = 0.0, comp = 0.0;
    for (int64_t d = 0; d <= delta; ++d) {
        uint64_t lo = hist_lo[d], hi = hist_hi ? hist_hi[d] : 0;
        if (lo == 0 && hi == 0) continue;
        double w = (double)L / (double)(L - d);
        double x = u128_to_double(lo, hi) * w;
        double s2 = sum + x;
        if (fabs(sum) >= fabs(x)) comp += (sum - s2) + x;
        else comp += (x - s2) + sum;
        sum = s2;
    }
    return (sum + comp) / p;
}

/* ---------------------------------------------------------------- estimate */

/*
 * Algorithm 1 with b = 1 and q_j = p for every window.
 *
 * Inputs: graph (m, src, dst, t), motif, delta >= 1, c >= 2, p in (0, 1],
 * seed.  force_shift: INT64_MIN for the random shift, otherwise a value in
 * {-c delta + 1, ..., 0} used in place of the draw (test hook for the
 * conditional-variance lemma).
 * Outputs: *s_out, *J_out, *nkept_out; kept window ids (1-based, ascending)
 * and their 64-bit counts into kept_ids / win_counts (first kept_cap of them;
 * either may be NULL); hist (delta+1 bins, nullable, cleared here) gets
 * N(Delta) summed over kept windows; *Z_out the estimate.
 */
int orc_estimate(int64_t m, const int32_t *src, const int32_t *dst, const int64_t *t,
                 int l, const int32_t *ms, const int32_t *md, int64_t delta,
                 int64_t cwin, double p, uint64_t seed, int64_t force_shift,
                 int64_t *s_out, int64_t *J_out, int64_t *nkept_out,
                 int64_t *kept_ids, uint64_t *win_counts, int64_t kept_cap,
                 uint64_t *hist, double *Z_out) {
    int k;
    if (m < 0 || delta < 1 || cwin < 2 || !(p > 0.0 && p <= 1.0) || !motif_ok(l, ms, md, &k))
        return ORC_EINVAL;
    if (delta > INT64_MAX / cwin) return ORC_EINVAL;
    int64_t L = cwin * delta;
    uint64_t *h = hist;
    uint64_t *own = NULL;
    if (!h) {
        own = (uint64_t *)calloc((size_t)delta + 1, sizeof(uint64_t));
        if (!own) return ORC_ENOMEM;
        h = own;
    } else {
        memset(h, 0, ((size_t)delta + 1) * sizeof(uint64_t));
    }
    /* normalise times to start at 0 */
    int64_t *tn = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
    if (!tn) { free(own); return ORC_ENOMEM; }
    int64_t tmin = 0, tmax = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (i == 0 || t[i] < tmin) tmin = t[i];
    }
    for (int64_t i = 0; i < m; ++i) {
        tn[i] = t[i] - tmin;
        if (tn[i] > tmax) tmax = tn[i];
    }
    int64_t J = 1 + (tmax / L) + ((tmax % L) ? 1 : 0);
    int64_t s;
    if (force_shift != INT64_MIN) {
        if (force_shift > 0 || force_shift <= -L) { free(tn); free(own); return ORC_EINVAL; }
        s = force_shift;
    } else {
        uint64_t x0 = orc_draw(seed, 0, 0, 0);
        s = -(int64_t)(x0 % (uint64_t)L);
    }
    int64_t nkept = 0;
    int rc = ORC_OK;
    for (int64_t j = 1; j <= J; ++j) {
        uint64_t x = orc_draw(seed, (uint64_t)j, 0, 1);
        double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);
        if (!(u < p)) continue;
        int64_t lo = s + (j - 1) * L;
        int64_t hi = s + j * L - 1;
        uint64_t tl, th;
        int r = orc_count(m, src, dst, tn, l, ms, md, delta, lo, hi, h, &tl, &th);
        if (r != ORC_OK) rc = r;
        if (th) rc = ORC_EOVERFLOW;
        if (nkept < kept_cap) {
            if (kept_ids) kept_ids[nkept] = j;
            if (win_counts) win_counts[nkept] = tl;
        }
        ++nkept;
    }
    *s_out = s;
    *J_out = J;
    *nkept_out = nkept;
    *Z_out = orc_weight(h, NULL, delta, L, p);
    free(tn);
    free(own);
    return rc;
}

/* ------------------------------------------------- edge-proportional q_j */

/* Neumaier step: sum += x with the running compensation comp. */
static void neu_add(double *sum, double *comp, double x) {
    double s2 = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - s2) + x;
    else *comp += (x - s2) + *sum;
    *sum = s2;
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* number of sorted values in [lo, hi] */
static int64_t count_in(const int64_t *v, int64_t n, int64_t lo, int64_t hi) {
    int64_t a = 0, b = n;
    while (a < b) { int64_t mid = a + (b - a) / 2; if (v[mid] < lo) a = mid + 1; else b = mid; }
    int64_t first = a;
    a = first; b = n;
    while (a < b) { int64_t mid = a + (b - a) / 2; if (v[mid] <= hi) a = mid + 1; else b = mid; }
    return a - first;
}

/*
 * Algorithm 1 with b shifts and the sampling probabilities the paper uses
 * (Sec. 4, "Choosing the sampling probabilities", equation heuristic_q):
 * q_j proportional to the number of temporal edges in window I_j,
 * q_j = min(1, r |T_j| / |T|), where |T| = m counts every edge of the graph
 * and a q_j above 1 is clamped (the sum stays unbiased with the clamped
 * value).  For shift k = 0 .. b-1: s_k from the draw (0, k, domain 0) (or
 * force_shift), window j kept when the uniform from draw (j, k, domain 1) is
 * below q_j; a kept window adds Y_{s,j} / q_j to Z_k, where
 * Y_{s,j} = sum over its instances of 1 / (1 - Delta / (c delta)) (the
 * weighted count w(I_j) of Sec. 4), taken from the window's own duration
 * histogram in ascending Delta.  Z = (1/b) sum_k Z_k.  Sums over Delta, over
 * kept windows (ascending j) and over shifts use Neumaier compensation.
 *
 * Outputs: *nkept_out (over all shifts); for the first cap kept windows, in
 * order of (k, j): win_k, win_j (1-based), win_q, win_y (any may be NULL);
 * *Z_out.
 */
int orc_estimate_q(int64_t m, const int32_t *src, const int32_t *dst, const int64_t *t,
                   int l, const int32_t *ms, const int32_t *md, int64_t delta,
                   int64_t cwin, double r, int32_t b, uint64_t seed, int64_t force_shift,
                   int64_t *nkept_out, int64_t *win_k, int64_t *win_j, double *win_q,
                   double *win_y, int64_t cap, double *Z_out) {
    int k;
    if (m < 0 || delta < 1 || cwin < 2 || !(r > 0.0) || b < 1 || !motif_ok(l, ms, md, &k))
        return ORC_EINVAL;
    if (delta > INT64_MAX / cwin) return ORC_EINVAL;
    const int64_t L = cwin * delta;
    int64_t *tn = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
    int64_t *ts = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
    uint64_t *h = (uint64_t *)calloc((size_t)delta + 1, sizeof(uint64_t));
    if (!tn || !ts || !h) { free(tn); free(ts); free(h); return ORC_ENOMEM; }
    int64_t tmin = 0, tmax = 0;
    for (int64_t i = 0; i < m; ++i)
        if (i == 0 || t[i] < tmin) tmin = t[i];
    for (int64_t i = 0; i < m; ++i) {
        tn[i] = t[i] - tmin;
        if (tn[i] > tmax) tmax = tn[i];
        ts[i] = tn[i];
    }
    qsort(ts, (size_t)m, sizeof(int64_t), cmp_i64);
    if (force_shift != INT64_MIN && (force_shift > 0 || force_shift <= -L)) {
        free(tn); free(ts); free(h);
        return ORC_EINVAL;
    }
    const int64_t J = 1 + (tmax / L) + ((tmax % L) ? 1 : 0);
    int rc = ORC_OK;
    int64_t nkept = 0;
    double zsum = 0.0, zcomp = 0.0;
    for (int32_t kk = 0; kk < b; ++kk) {
        int64_t s = force_shift;
        if (force_shift == INT64_MIN) s = -(int64_t)(orc_draw(seed, 0, (uint32_t)kk, 0) % (uint64_t)L);
        double zk = 0.0, zkc = 0.0;
        for (int64_t j = 1; j <= J; ++j) {
            const int64_t lo = s + (j - 1) * L, hi = s + j * L - 1;
            const int64_t tj = count_in(ts, m, lo, hi);
            double q = r * (double)tj / (double)(m ? m : 1);
            if (q > 1.0) q = 1.0;
            const uint64_t x = orc_draw(seed, (uint64_t)j, (uint32_t)kk, 1);
            const double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);
            if (!(u < q)) continue;
            memset(h, 0, ((size_t)delta + 1) * sizeof(uint64_t));
            uint64_t cl, ch;
            int rr = orc_count(m, src, dst, tn, l, ms, md, delta, lo, hi, h, &cl, &ch);
            if (rr != ORC_OK) rc = rr;
            const double y = orc_weight(h, NULL, delta, L, 1.0);
            neu_add(&zk, &zkc, y / q);
            if (nkept < cap) {
                if (win_k) win_k[nkept] = kk;
                if (win_j) win_j[nkept] = j;
                if (win_q) win_q[nkept] = q;
                if (win_y) win_y[nkept] = y;
            }
            ++nkept;
        }
        neu_add(&zsum, &zcomp, zk + zkc);
    }
    *nkept_out = nkept;
    *Z_out = (zsum + zcomp) / (double)b;
    free(tn);
    free(ts);
    free(h);
    return rc;
}
