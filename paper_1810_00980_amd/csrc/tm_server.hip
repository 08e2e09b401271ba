// Query server: continuous batching of count/estimate queries over
// device-resident graphs, admitted against a device-memory budget.
//
// A dispatcher thread keeps a FIFO of submitted queries.  Whenever a worker
// slot is free it takes the oldest query that fits the memory budget and
// merges every pending query that can share its device work: exact counts of
// three-edge motifs on the same graph and delta share one sweep; estimates of
// three-edge motifs on the same graph share one persistent launch sequence,
// whatever their motifs, deltas, c, p and seeds (each is its own estimator
// in the mixed batch; a lone one, or one on a heavy graph, takes the plain
// weighted sweep, and a lone triangle estimate may sum its triangles over the
// graph's static triangles, found when the graph was added).  It reserves
// the batch's device workspace from the budget and hands the batch to the
// slot.  The static triangles' per-call workspace depends on the query's
// windows and is only known on the device, so that path asks the slot for it
// step by step before it allocates: what fits the budget then is added to the
// batch's charge, and otherwise the estimate counts its triangles over the
// incidence lists.  Each slot is a host thread with its own
// HIP stream (default priority), so batches on different slots overlap on the
// device; finishing a batch returns its workspace to the budget and wakes the
// dispatcher, which admits waiting queries as memory and slots free up.
// Batches on the heavy graphs (an eighth or more of the largest graph's
// edges, when lighter graphs are resident too) take at most half the slots:
// a heavy query fills the device by itself, so more of them at once only
// stretch each other, while the queries on small graphs would wait behind
// them.
//
// A batch is charged the device bytes its path allocates (every buffer of
// that path, at the sizes the graph and queries fix, with upper bounds where
// a size is only known on the device); the bytes it really allocated are
// measured (DevTally) and reported beside the charge.  A slot thread keeps
// its grow-only workspaces between batches (a free is a device-wide
// synchronisation that would stall the other slots), and what it holds is
// measured after each batch and counted against the budget as well; when the
// oldest query does not fit, an idle slot is asked to free what it holds.  A
// query whose workspace alone exceeds the budget is completed with
// TM_EBUDGET.  Results do not depend on how queries were batched: every
// count is an exact integer and every estimate is computed from exact
// integer sums.
#include "tm_common.h"

#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

struct tm_server;

namespace {

using Clock = std::chrono::steady_clock;

struct Pending {
    int64_t ticket;
    tm_query q;
    Clock::time_point submit;
};

constexpr size_t TM_SERVER_MAX_BATCH = 256;
int64_t buf(int64_t b) { return b > 0 ? b : 256; }  // DevBuf's size for a request of b bytes

// Device bytes of the path a batch takes (the DevBufs it allocates, alive
// together).  All queries of a batch share graph and kind; a batch of more
// than one query holds three-edge motifs only.
// whether a batch of these queries may take the static triangles: one
// estimate of a triangle motif on a graph whose static triangles are kept
bool static_candidate(const tm_graph *g, const std::vector<tm_query> &b) {
    if (b.size() != 1 || b[0].kind != 1) return false;
    const int c = tm_sweep_code_of(&b[0].motif);
    return c >= 20 && c < 28 && tm_tri_static_kept(g);
}

int64_t batch_ws_bytes(const tm_graph *g, const std::vector<tm_query> &b) {
    const tm_query &q0 = b[0];
    const bool three = tm_sweep_code_of(&q0.motif) >= 0;
    const int64_t m1 = g->m > 0 ? g->m : 1;
    if (q0.kind == 0) {
        if (three) {
            // the sweep's accumulators and work counters, and the exact
            // triangle sweep's claim order when a triangle motif is asked for
            int64_t bytes = buf(36 * 4 * 8) + buf(TM_SWEEP_COUNTER_BYTES);
            for (const tm_query &q : b) {
                const int c = tm_sweep_code_of(&q.motif);
                if (c >= 20 && c < 28) {
                    bytes += tm_tri_order_bytes(g);
                    break;
                }
            }
            return bytes;
        }
        uint32_t d[4];
        if (tm_star4_shape(&q0.motif, d)) return tm_star4_bytes(g, 0) + tm_star4_build_bytes(g);
        // the generic counter over every edge
        return buf(64) + tm_generic_bytes(g->m, q0.motif.l);
    }
    if (three && b.size() == 1) {
        // the plain weighted sweep: accumulators, work counters, weights (the
        // static triangles' workspace is granted while the batch runs)
        return buf(36 * 4 * 8) + buf(TM_SWEEP_COUNTER_BYTES) + buf((q0.delta + 1) * 8);
    }
    if (three) {
        std::vector<int64_t> delta, L;
        for (const tm_query &q : b) {
            delta.push_back(q.delta);
            L.push_back(q.c * q.delta);
        }
        return tm_batch_mixed_bytes(g, (int64_t)b.size(), delta.data(), L.data());
    }
    uint32_t d[4];
    if (tm_star4_shape(&q0.motif, d)) return tm_star4_bytes(g, q0.delta) + tm_star4_build_bytes(g);
    // the generic estimate with diagnostics: kept-anchor lists (the kept
    // anchors are at most m), the duration histogram, per-window totals, the
    // generic counter's items, the window list and the scan workspace
    const int64_t L = q0.c * q0.delta;
    const int64_t J = 1 + g->t_span / L + ((g->t_span % L) ? 1 : 0);
    int64_t bytes = buf(64) + 3 * buf(8 * m1) + 6 * buf(8 * m1) + buf(4 * m1);
    bytes += buf(16 * (q0.delta + 1)) + buf((2 + 2 * m1) * 8 + 64);
    bytes += tm_generic_bytes(m1, q0.motif.l);
    if (J <= ((int64_t)1 << 24)) bytes += 2 * buf(8 * J) + buf(8) + buf(8);
    bytes += tm_scan_ws_bytes(m1 > J ? m1 : J);
    return bytes;
}

// heavy: the graph of the query is heavy (see tm_server::is_heavy)
bool shareable(const tm_query &a, const tm_query &b, bool heavy) {
    if (a.graph != b.graph || a.kind != b.kind) return false;
    if (tm_sweep_code_of(&a.motif) < 0 || tm_sweep_code_of(&b.motif) < 0) return false;
    if (a.kind == 0) return a.delta == b.delta;  // one sweep counts all
    // estimates: one estimator each in the mixed batch, which saves launches
    // and host round trips; on a heavy graph each estimator's own work
    // dominates, and the plain sweep of each serves them as well
    return !heavy;
}

}  // namespace

struct tm_server {
    std::mutex mu;
    std::condition_variable cv_disp, cv_done;
    std::deque<Pending> queue;
    std::map<int64_t, tm_result> done;  // finished, not yet collected
    std::vector<uint8_t> state;         // per ticket: 0 pending, 1 ready, 2 collected
    std::vector<const tm_graph *> graphs;
    std::vector<std::thread> workers;
    std::thread dispatcher;
    std::vector<std::vector<Pending>> slot_work;
    std::vector<int64_t> slot_bytes;   // charge of the running batch
    std::vector<int64_t> slot_held;    // device bytes the slot thread holds between batches
    std::vector<bool> release_req;     // asked to free what it holds
    std::vector<hipStream_t> streams;
    std::vector<bool> slot_busy;
    std::vector<bool> slot_heavy;      // the running batch is on a heavy graph
    std::vector<bool> slot_static;     // the running batch may take the static triangles
    std::vector<int64_t> slot_granted; // of the charge, what the static triangles were granted
    // heavy: at least an eighth of the edges of the largest graph added,
    // when some graph is lighter than that (one size class: none is heavy)
    bool is_heavy(const tm_graph *g) const {
        int64_t mx = 0;
        for (const tm_graph *h : graphs) mx = std::max<int64_t>(mx, h->m);
        bool any_light = false;
        for (const tm_graph *h : graphs) any_light = any_light || 8 * h->m < mx;
        return any_light && 8 * g->m >= mx;
    }
    std::condition_variable cv_slot;
    int64_t budget = 0, in_use = 0, peak = 0, next_ticket = 1;
    int64_t submitted = 0, completed = 0, rejected = 0, batches = 0;
    int64_t measured_max = 0, over_charge = 0;
    bool stop = false, have_first = false;
    Clock::time_point first_submit, last_done;
    std::vector<double> lat_ms;
    double edges_done = 0;
    int device = 0;

    void finish_query(const Pending &pq, const tm_result &r) {
        done[pq.ticket] = r;
        state[(size_t)pq.ticket] = 1;
        ++completed;
        if (r.status == TM_OK) {
            lat_ms.push_back(r.latency_ms);
            edges_done += (double)graphs[(size_t)pq.q.graph]->m;
        } else {
            ++rejected;
        }
        last_done = Clock::now();
    }

    void dispatch_loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            cv_disp.wait(lk, [&] {
                if (stop) return true;
                if (queue.empty()) return false;
                for (bool b : slot_busy)
                    if (!b) return true;
                return false;
            });
            if (stop && queue.empty()) return;
            if (stop) {
                // drain: fail what is left
                while (!queue.empty()) {
                    tm_result r;
                    memset(&r, 0, sizeof r);
                    r.status = TM_EDEVICE;
                    finish_query(queue.front(), r);
                    queue.pop_front();
                }
                cv_done.notify_all();
                return;
            }
            int slot = -1;
            for (size_t i = 0; i < slot_busy.size(); ++i)
                if (!slot_busy[i]) {
                    slot = (int)i;
                    break;
                }
            // oldest admissible query: first in FIFO whose workspace fits;
            // a query on a heavy graph waits while half the slots run heavy
            // batches, so that queries on the small graphs keep slots
            int heavy_running = 0;
            for (size_t k = 0; k < slot_busy.size(); ++k) heavy_running += slot_busy[k] && slot_heavy[k];
            const int heavy_cap = std::max<int>(1, (int)slot_busy.size() / 2);
            bool admitted = false;
            for (size_t qi = 0; qi < queue.size(); ++qi) {
                const Pending &head = queue[qi];
                const tm_graph *g = graphs[(size_t)head.q.graph];
                const bool heavy = is_heavy(g);
                if (heavy && heavy_running >= heavy_cap) continue;
                int64_t need = batch_ws_bytes(g, {head.q});
                bool use_static = static_candidate(g, {head.q});
                if (need > budget) {
                    tm_result r;
                    memset(&r, 0, sizeof r);
                    r.status = TM_EBUDGET;
                    finish_query(head, r);
                    queue.erase(queue.begin() + (long)qi);
                    cv_done.notify_all();
                    admitted = true;  // re-evaluate
                    break;
                }
                if (in_use + need > budget) {
                    // ask idle slots that hold workspaces to free them
                    for (size_t k = 0; k < slot_busy.size(); ++k)
                        if (!slot_busy[k] && slot_held[k] > 0 && !release_req[k]) {
                            release_req[k] = true;
                            cv_slot.notify_all();
                        }
                    continue;
                }
                std::vector<Pending> batch;
                std::vector<tm_query> bq;
                batch.push_back(head);
                bq.push_back(head.q);
                queue.erase(queue.begin() + (long)qi);
                for (size_t k = 0; k < queue.size();) {
                    bool take = batch.size() < TM_SERVER_MAX_BATCH && shareable(batch[0].q, queue[k].q, heavy);
                    if (take) {
                        // a merged query must keep the batch within what is left
                        bq.push_back(queue[k].q);
                        const int64_t more = batch_ws_bytes(g, bq);
                        if (in_use + more > budget) {
                            bq.pop_back();
                            take = false;
                        } else {
                            need = more;
                            use_static = false;  // several queries take the mixed launch
                        }
                    }
                    if (take) {
                        batch.push_back(queue[k]);
                        queue.erase(queue.begin() + (long)k);
                    } else {
                        ++k;
                    }
                }
                in_use += need;
                peak = std::max(peak, in_use);
                slot_busy[(size_t)slot] = true;
                slot_heavy[(size_t)slot] = heavy;
                slot_static[(size_t)slot] = use_static;
                slot_bytes[(size_t)slot] = need;
                slot_work[(size_t)slot] = std::move(batch);
                ++batches;
                cv_slot.notify_all();
                admitted = true;
                break;
            }
            if (!admitted) {
                // nothing fits the budget now: wait until a batch returns memory
                cv_disp.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
    }

    void run_batch(int slot, std::vector<Pending> &batch) {
        hipStream_t st = streams[(size_t)slot];
        const int64_t base = t_dev_tally.live;
        t_dev_tally.peak = base;
        const tm_query &q0 = batch[0].q;
        const tm_graph *g = graphs[(size_t)q0.graph];
        Clock::time_point start = Clock::now();
        std::vector<tm_result> res(batch.size());
        for (auto &r : res) memset(&r, 0, sizeof r);
        int n = (int)batch.size();
        std::vector<tm_motif> ms((size_t)n);
        for (int i = 0; i < n; ++i) ms[(size_t)i] = batch[(size_t)i].q.motif;
        if (q0.kind == 0) {
            std::vector<tm_u128> cnt((size_t)n);
            tm_status s = n > 1 ? tm_count_exact_multi(g, n, ms.data(), q0.delta, cnt.data(), nullptr, nullptr, st)
                                : tm_count_exact(g, &ms[0], q0.delta, &cnt[0], st);
            for (int i = 0; i < n; ++i) {
                res[(size_t)i].status = s;
                res[(size_t)i].count = cnt[(size_t)i];
            }
        } else {
            std::vector<double> est((size_t)n);
            std::vector<tm_u128> kc((size_t)n);
            std::vector<tm_est_query> eq((size_t)n);
            for (int i = 0; i < n; ++i) {
                const tm_query &q = batch[(size_t)i].q;
                eq[(size_t)i] = tm_est_query{q.motif, q.delta, q.c, q.p, q.seed};
            }
            // a lone three-edge estimate takes the plain sweep; several share
            // one mixed launch sequence, enqueued on the slot's stream (a
            // graph captured per batch would be replayed once, and a capture
            // must not overlap the other slots' runtime calls)
            tm_status s = (n == 1 && tm_sweep_code_of(&eq[0].motif) >= 0)
                              ? tm_estimate_multi(g, 1, &eq[0].motif, eq[0].delta, eq[0].c, eq[0].p, eq[0].seed,
                                                  est.data(), kc.data(), st)
                              : tm_estimate_mixed_ex(g, n, eq.data(), est.data(), kc.data(), st, false);
            for (int i = 0; i < n; ++i) {
                res[(size_t)i].status = s;
                res[(size_t)i].estimate = est[(size_t)i];
                res[(size_t)i].count = kc[(size_t)i];
            }
        }
        Clock::time_point end = Clock::now();
        const int64_t measured = t_dev_tally.peak - base;
        std::lock_guard<std::mutex> lk(mu);
        const int64_t charged = slot_bytes[(size_t)slot];  // with what the static triangles were granted
        measured_max = std::max(measured_max, measured);
        if (measured > charged) ++over_charge;
        for (int i = 0; i < n; ++i) {
            tm_result &r = res[(size_t)i];
            r.ws_charged = charged;
            r.ws_measured = measured;
            r.latency_ms = std::chrono::duration<double, std::milli>(end - batch[(size_t)i].submit).count();
            r.queue_ms = std::chrono::duration<double, std::milli>(start - batch[(size_t)i].submit).count();
            r.batch_size = n;
            r.slot = slot;
            finish_query(batch[(size_t)i], r);
        }
        cv_done.notify_all();
    }

    // The static triangles' set-up on a slot thread asks for the bytes its
    // call allocates in all: the part beyond what the batch was granted so
    // far is added to the batch's charge when it fits the budget.
    struct GrantCtx {
        tm_server *S;
        int slot;
    };
    static bool grant(void *ctx, int64_t bytes) {
        const GrantCtx *c = static_cast<const GrantCtx *>(ctx);
        tm_server *S = c->S;
        std::lock_guard<std::mutex> lk(S->mu);
        const size_t k = (size_t)c->slot;
        const int64_t more = bytes - S->slot_granted[k];
        if (more <= 0) return true;
        if (S->in_use + more > S->budget) return false;
        S->in_use += more;
        S->slot_bytes[k] += more;
        S->slot_granted[k] = bytes;
        S->peak = std::max(S->peak, S->in_use);
        return true;
    }

    // what this slot thread holds now replaces what it held (lock held)
    void set_held(int slot) {
        const int64_t h = std::max<int64_t>(0, t_dev_tally.live);
        in_use += h - slot_held[(size_t)slot];
        slot_held[(size_t)slot] = h;
        peak = std::max(peak, in_use);
    }

    void worker_loop(int slot) {
        (void)hipSetDevice(device);
        t_dev_tally.live = t_dev_tally.peak = 0;  // this thread's own allocations only
        GrantCtx gc{this, slot};
        tm_tri_static_set_grant(&tm_server::grant, &gc);  // a batch allocates no more than it was charged
        while (true) {
            std::vector<Pending> batch;
            bool use_static = false;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_slot.wait(lk, [&] {
                    return stop || !slot_work[(size_t)slot].empty() || release_req[(size_t)slot];
                });
                if (release_req[(size_t)slot] && slot_work[(size_t)slot].empty()) {
                    lk.unlock();
                    tm_release_thread_ws();
                    lk.lock();
                    release_req[(size_t)slot] = false;
                    set_held(slot);
                    cv_disp.notify_all();
                    continue;
                }
                if (slot_work[(size_t)slot].empty()) return;  // stop requested, no work
                batch = std::move(slot_work[(size_t)slot]);
                slot_work[(size_t)slot].clear();
                use_static = slot_static[(size_t)slot];
            }
            tm_tri_static_enable(use_static);
            run_batch(slot, batch);
            {
                std::lock_guard<std::mutex> lk(mu);
                in_use -= slot_bytes[(size_t)slot];
                slot_bytes[(size_t)slot] = 0;
                slot_granted[(size_t)slot] = 0;
                set_held(slot);
                slot_busy[(size_t)slot] = false;
            }
            cv_disp.notify_all();
        }
    }
};

extern "C" tm_status tm_server_create(int32_t slots, int64_t budget_bytes, tm_server **out) {
    if (!out || slots < 1 || slots > 64 || budget_bytes <= 0) return TM_EINVAL;
    tm_server *S = new (std::nothrow) tm_server();
    if (!S) return TM_ENOMEM;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return TM_EDEVICE;
    }
    S->budget = budget_bytes;
    S->slot_work.resize((size_t)slots);
    S->slot_bytes.assign((size_t)slots, 0);
    S->slot_held.assign((size_t)slots, 0);
    S->release_req.assign((size_t)slots, false);
    S->slot_busy.assign((size_t)slots, false);
    S->slot_heavy.assign((size_t)slots, false);
    S->slot_static.assign((size_t)slots, false);
    S->slot_granted.assign((size_t)slots, 0);
    for (int i = 0; i < slots; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t s2 : S->streams) (void)hipStreamDestroy(s2);
            delete S;
            return TM_EDEVICE;
        }
        S->streams.push_back(st);
    }
    for (int i = 0; i < slots; ++i) S->workers.emplace_back([S, i] { S->worker_loop(i); });
    S->dispatcher = std::thread([S] { S->dispatch_loop(); });
    *out = S;
    return TM_OK;
}

extern "C" tm_status tm_server_add_graph(tm_server *S, const tm_graph *g, int32_t *graph_id) {
    if (!S || !g || !graph_id) return TM_EINVAL;
    // the static triangles of a large graph, found here once (their search's
    // temporaries are not any batch's), so that lone triangle estimates can
    // sum over them
    bool kept = false;
    TM_TRY(tm_tri_static_prepare(const_cast<tm_graph *>(g), nullptr, &kept));
    TM_HIP(hipStreamSynchronize(nullptr));
    std::lock_guard<std::mutex> lk(S->mu);
    S->graphs.push_back(g);
    *graph_id = (int32_t)S->graphs.size() - 1;
    return TM_OK;
}

extern "C" tm_status tm_server_submit(tm_server *S, const tm_query *q, int64_t *ticket) {
    if (!S || !q || !ticket) return TM_EINVAL;
    MotifPlan P;
    TM_TRY(tm_make_plan(&q->motif, &P));
    if (q->kind != 0 && q->kind != 1) return TM_EINVAL;
    if (q->delta < 0 || (q->kind == 1 && (q->delta < 1 || q->c < 2 || !(q->p > 0.0 && q->p <= 1.0))))
        return TM_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (q->graph < 0 || (size_t)q->graph >= S->graphs.size()) return TM_EINVAL;
    Pending pq;
    pq.ticket = S->next_ticket++;
    S->state.resize((size_t)S->next_ticket, 0);
    pq.q = *q;
    pq.submit = Clock::now();
    if (!S->have_first) {
        S->first_submit = pq.submit;
        S->have_first = true;
    }
    S->queue.push_back(pq);
    ++S->submitted;
    *ticket = pq.ticket;
    S->cv_disp.notify_all();
    return TM_OK;
}

extern "C" tm_status tm_server_wait(tm_server *S, int64_t ticket, tm_result *res) {
    if (!S || !res) return TM_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    if (ticket <= 0 || ticket >= S->next_ticket) return TM_EINVAL;
    if (S->state[(size_t)ticket] == 2) return TM_EINVAL;  // already collected
    S->cv_done.wait(lk, [&] { return S->state[(size_t)ticket] != 0; });
    if (S->state[(size_t)ticket] == 2) return TM_EINVAL;  // collected by another waiter
    auto it = S->done.find(ticket);
    *res = it->second;
    S->done.erase(it);
    S->state[(size_t)ticket] = 2;
    return TM_OK;
}

extern "C" tm_status tm_server_stats_get(tm_server *S, tm_server_stats *out) {
    if (!S || !out) return TM_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    memset(out, 0, sizeof *out);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->rejected = S->rejected;
    out->batches = S->batches;
    out->budget_bytes = S->budget;
    out->peak_bytes = S->peak;
    out->measured_max_bytes = S->measured_max;
    out->over_charge = S->over_charge;
    out->uncollected = (int64_t)S->done.size();
    std::vector<double> v = S->lat_ms;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double f) {
            // nearest-rank percentile
            size_t r = (size_t)std::ceil(f * (double)v.size());
            if (r < 1) r = 1;
            return v[r - 1];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        double s = 0;
        for (double x : v) s += x;
        out->mean_ms = s / (double)v.size();
    }
    if (S->have_first && S->completed > 0) {
        out->wall_s = std::chrono::duration<double>(S->last_done - S->first_submit).count();
        out->edges_per_s = out->wall_s > 0 ? S->edges_done / out->wall_s : 0;
    }
    return TM_OK;
}

extern "C" void tm_server_destroy(tm_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_disp.notify_all();
    S->cv_slot.notify_all();
    if (S->dispatcher.joinable()) S->dispatcher.join();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->cv_slot.notify_all();
    }
    for (auto &w : S->workers)
        if (w.joinable()) w.join();
    for (hipStream_t st : S->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    delete S;
}
