// Query server: continuous batching of count/estimate queries over
// device-resident graphs, admitted against a device-memory budget.
//
// A dispatcher thread keeps a FIFO of submitted queries.  Whenever a worker
// slot is free it takes the oldest query, merges every pending query that
// can share its device pass (exact counts of three-edge motifs on the same
// graph and delta share one sweep; estimates of three-edge motifs with the
// same graph, delta, c, p and seed share one windowed sweep, because the
// shift and kept windows depend only on those), reserves the batch's
// workspace from the budget, and hands the batch to the slot.  Each slot is a
// host thread with its own HIP stream (default priority), so batches on
// different slots overlap on the device; finishing a batch returns its
// workspace to the budget and wakes the dispatcher, which admits waiting
// queries as memory and slots free up.  A query whose workspace alone exceeds
// the budget is completed with TM_EBUDGET.  Results do not depend on how
// queries were batched: every count is an exact integer and every estimate
// is computed from exact integer sums.
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

struct Done {
    tm_result r;
    bool ready = false;
    bool claimed = false;
};

int64_t query_ws_bytes(const tm_graph *g, const tm_query &q) {
    bool three = tm_sweep_code_of(&q.motif) >= 0;
    if (three) return 36 * 4 * 8 + 64 + (q.kind == 1 ? (q.delta + 1) * 8 : 0);
    // generic path: kept-anchor lists (8 arrays of m words) and a histogram
    return 8 * 8 * g->m + 16 * (q.delta + 1) + 4096;
}

bool shareable(const tm_query &a, const tm_query &b) {
    if (a.graph != b.graph || a.kind != b.kind || a.delta != b.delta) return false;
    if (tm_sweep_code_of(&a.motif) < 0 || tm_sweep_code_of(&b.motif) < 0) return false;
    if (a.kind == 0) return true;
    return a.c == b.c && a.p == b.p && a.seed == b.seed;
}

}  // namespace

struct tm_server {
    std::mutex mu;
    std::condition_variable cv_disp, cv_done;
    std::deque<Pending> queue;
    std::map<int64_t, Done> done;
    std::vector<const tm_graph *> graphs;
    std::vector<std::thread> workers;
    std::thread dispatcher;
    std::vector<std::vector<Pending>> slot_work;
    std::vector<int64_t> slot_bytes;
    std::vector<hipStream_t> streams;
    std::vector<bool> slot_busy;
    std::condition_variable cv_slot;
    int64_t budget = 0, in_use = 0, peak = 0, next_ticket = 1;
    int64_t submitted = 0, completed = 0, rejected = 0, batches = 0;
    bool stop = false, have_first = false;
    Clock::time_point first_submit, last_done;
    std::vector<double> lat_ms;
    double edges_done = 0;
    int device = 0;

    void finish_query(const Pending &pq, const tm_result &r) {
        Done &d = done[pq.ticket];
        d.r = r;
        d.ready = true;
        d.claimed = false;
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
            // oldest admissible query: first in FIFO whose workspace fits
            bool admitted = false;
            for (size_t qi = 0; qi < queue.size(); ++qi) {
                const Pending &head = queue[qi];
                const tm_graph *g = graphs[(size_t)head.q.graph];
                int64_t need = query_ws_bytes(g, head.q);
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
                if (in_use + need > budget) continue;
                std::vector<Pending> batch;
                batch.push_back(head);
                queue.erase(queue.begin() + (long)qi);
                for (size_t k = 0; k < queue.size();) {
                    if (batch.size() < 36 && shareable(batch[0].q, queue[k].q)) {
                        batch.push_back(queue[k]);
                        queue.erase(queue.begin() + (long)k);
                    } else {
                        ++k;
                    }
                }
                in_use += need;
                peak = std::max(peak, in_use);
                slot_busy[(size_t)slot] = true;
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
            tm_status s;
            if (n > 1) {
                s = tm_estimate_multi(g, n, ms.data(), q0.delta, q0.c, q0.p, q0.seed, est.data(), kc.data(), st);
            } else {
                tm_est_info info;
                memset(&info, 0, sizeof info);
                bool three = tm_sweep_code_of(&ms[0]) >= 0;
                s = three ? tm_estimate_multi(g, 1, ms.data(), q0.delta, q0.c, q0.p, q0.seed, est.data(), kc.data(), st)
                          : tm_estimate(g, &ms[0], q0.delta, q0.c, q0.p, q0.seed, &est[0], &info, st);
                if (!three) kc[0] = info.kept_count;
            }
            for (int i = 0; i < n; ++i) {
                res[(size_t)i].status = s;
                res[(size_t)i].estimate = est[(size_t)i];
                res[(size_t)i].count = kc[(size_t)i];
            }
        }
        Clock::time_point end = Clock::now();
        std::lock_guard<std::mutex> lk(mu);
        for (int i = 0; i < n; ++i) {
            tm_result &r = res[(size_t)i];
            r.latency_ms = std::chrono::duration<double, std::milli>(end - batch[(size_t)i].submit).count();
            r.queue_ms = std::chrono::duration<double, std::milli>(start - batch[(size_t)i].submit).count();
            r.batch_size = n;
            r.slot = slot;
            finish_query(batch[(size_t)i], r);
        }
        cv_done.notify_all();
    }

    void worker_loop(int slot) {
        (void)hipSetDevice(device);
        while (true) {
            std::vector<Pending> batch;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_slot.wait(lk, [&] { return stop || !slot_work[(size_t)slot].empty(); });
                if (slot_work[(size_t)slot].empty()) return;  // stop requested, no work
                batch = std::move(slot_work[(size_t)slot]);
                slot_work[(size_t)slot].clear();
            }
            run_batch(slot, batch);
            {
                std::lock_guard<std::mutex> lk(mu);
                in_use -= slot_bytes[(size_t)slot];
                slot_bytes[(size_t)slot] = 0;
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
    S->slot_busy.assign((size_t)slots, false);
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
    auto it0 = S->done.find(ticket);
    if (it0 != S->done.end() && it0->second.claimed) return TM_EINVAL;  // already collected
    S->cv_done.wait(lk, [&] {
        auto it = S->done.find(ticket);
        return it != S->done.end() && it->second.ready;
    });
    Done &d = S->done[ticket];
    d.claimed = true;
    *res = d.r;
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
