// Serving: graphs stay resident in HBM; count queries with any deltas and windows are submitted
// from any thread and answered by continuous batching.
//
// One worker thread owns kSlots batch runners (each with its own stream, tables and scratch).
// Whenever a runner is free and queries are waiting, the worker takes up to max_batch of them and
// launches them as one batched launch on that runner; queries that arrive while batches are on
// the device go into the next batch, which runs alongside them.  Completed batches hand each
// query its counts and wake its waiter.  Graphs are admitted against the server's HBM budget;
// a query past its deadline before it reaches the device completes with DT_ETIMEDOUT; an invalid
// query is refused at submission without touching the others.
#include <chrono>
#include <unordered_map>

#include "internal.h"

namespace dt {

uint64_t graph_device_bytes(const dt_graph *g) {
    const DevMem *ms[] = {&g->sx, &g->sy, &g->row, &g->col, &g->ceid, &g->psid, &g->pdir, &g->pkey,
                          &g->pstart, &g->c1, &g->core, &g->rank, &g->order, &g->dag_row, &g->dag_col,
                          &g->eoff, &g->key, &g->sched.light, &g->sched.medium, &g->sched.mitems,
                          &g->sched.light_w, &g->sched.medium_w, &g->sched.mitems_w, &g->sched.heavy,
                          &g->sched.hslot, &g->sched.chunks, &g->sched.pchunks, &g->sched.mlev_w,
                          &g->sched.unit};
    uint64_t b = 0;
    for (const DevMem *m : ms) b += m->bytes;
    // scratch of the heavy path, taken per query in flight
    b += g->sched.n_slots * 8 * sizeof(int64_t) + g->sched.n_pchunks * 8 * sizeof(int64_t) + 48 * g->sched.n_heavy;
    return b;
}

namespace {

constexpr int kSlots = 3;

struct Ticket {
    bool done = false;
    int rc = DT_OK;
    int64_t out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t gid = 0;
    DQuery q{};
    bool empty = false;
    std::chrono::steady_clock::time_point submitted;
};

struct Slot {
    BatchRunner *runner = nullptr;
    bool busy = false;
    std::vector<uint64_t> tickets;
    std::vector<dt_graph *> graphs;
    std::vector<DQuery> qs;
    std::unique_ptr<bool[]> empty;
    size_t cap = 0;
};

}  // namespace
}  // namespace dt

struct dt_server {
    dt_ctx *ctx = nullptr;
    dt_server_cfg cfg{};
    uint64_t budget = 0, used = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<dt_graph *> graphs;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, dt::Ticket> tickets;
    uint64_t next_ticket = 1;
    uint32_t inflight = 0;
    bool stopping = false;
    int worker_rc = DT_OK;
    dt::Slot slots[dt::kSlots];
    std::thread worker;
};

namespace dt {
namespace {

void complete_slot(dt_server *s, Slot &sl) {
    // called without the lock: results are in the runner's pinned buffer once `done` fired
    const uint64_t k = sl.tickets.size();
    std::vector<int64_t> out(8 * k);
    int rc = batch_wait(sl.runner, k, sl.empty.get(), reinterpret_cast<int64_t(*)[8]>(out.data()));
    std::lock_guard<std::mutex> lk(s->mu);
    for (uint64_t i = 0; i < k; ++i) {
        auto it = s->tickets.find(sl.tickets[i]);
        if (it == s->tickets.end()) continue;
        Ticket &t = it->second;
        t.rc = rc;
        for (int j = 0; j < 8; ++j) t.out[j] = out[8 * i + j];
        t.done = true;
    }
    s->inflight -= (uint32_t)k;
    sl.busy = false;
    sl.tickets.clear();
    s->cv_done.notify_all();
}

void worker_main(dt_server *s) {
    (void)hipSetDevice(s->ctx->device);
    const uint32_t max_batch = s->cfg.max_batch ? s->cfg.max_batch : 512;
    const int64_t deadline = s->cfg.deadline_ns;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // 1. hand back finished batches
        bool progressed = false;
        for (Slot &sl : s->slots) {
            if (sl.busy && batch_ready(sl.runner)) {
                lk.unlock();
                complete_slot(s, sl);
                lk.lock();
                progressed = true;
            }
        }
        // 2. launch waiting queries on a free runner
        Slot *free_slot = nullptr;
        for (Slot &sl : s->slots)
            if (!sl.busy) { free_slot = &sl; break; }
        if (free_slot && !s->pending.empty()) {
            Slot &sl = *free_slot;
            sl.tickets.clear();
            sl.graphs.clear();
            sl.qs.clear();
            const auto now = std::chrono::steady_clock::now();
            while (!s->pending.empty() && sl.tickets.size() < max_batch) {
                uint64_t id = s->pending.front();
                s->pending.pop_front();
                Ticket &t = s->tickets[id];
                if (deadline > 0 &&
                    std::chrono::duration_cast<std::chrono::nanoseconds>(now - t.submitted).count() > deadline) {
                    t.rc = fail(DT_ETIMEDOUT, "query passed its deadline before reaching the device");
                    t.done = true;
                    s->inflight--;
                    s->cv_done.notify_all();
                    continue;
                }
                sl.tickets.push_back(id);
                sl.graphs.push_back(s->graphs[t.gid]);
                sl.qs.push_back(t.q);
            }
            const size_t k = sl.tickets.size();
            if (k) {
                if (sl.cap < k) {
                    sl.empty.reset(new bool[k]);
                    sl.cap = k;
                }
                for (size_t i = 0; i < k; ++i) sl.empty[i] = s->tickets[sl.tickets[i]].empty;
                sl.busy = true;
                lk.unlock();
                // item lengths for this batch's size class: cached, or tuned now on this batch
                BatchTune bt;
                int rc = batch_tuned(s->ctx, sl.runner, k, sl.graphs.data(), sl.qs.data(), sl.empty.get(), &bt);
                if (rc == DT_OK)
                    rc = batch_plan_and_launch(sl.runner, k, sl.graphs.data(), sl.qs.data(), sl.empty.get(), bt);
                lk.lock();
                if (rc != DT_OK) {
                    for (uint64_t id : sl.tickets) {
                        Ticket &t = s->tickets[id];
                        t.rc = rc;
                        t.done = true;
                    }
                    s->inflight -= (uint32_t)k;
                    sl.busy = false;
                    sl.tickets.clear();
                    s->cv_done.notify_all();
                }
            }
            progressed = true;
        }
        bool any_busy = false;
        for (Slot &sl : s->slots) any_busy |= sl.busy;
        if (s->stopping && s->pending.empty() && !any_busy) break;
        if (progressed) continue;
        if (any_busy) {
            bool all_busy = true;
            for (Slot &sl : s->slots) all_busy &= sl.busy;
            if (all_busy) {
                // nothing can start until a runner frees: wait for the oldest on the device
                Slot *first = nullptr;
                for (Slot &sl : s->slots)
                    if (sl.busy) { first = &sl; break; }
                lk.unlock();
                if (first) (void)batch_sync(first->runner);
                lk.lock();
            } else {
                s->cv_work.wait_for(lk, std::chrono::microseconds(50));
            }
        } else {
            s->cv_work.wait(lk, [s] { return s->stopping || !s->pending.empty(); });
        }
    }
}

}  // namespace
}  // namespace dt

using namespace dt;

extern "C" {

int dt_server_start(dt_ctx *ctx, const dt_server_cfg *cfg, dt_server **out) {
    clear_error();
    if (!ctx || !out) return fail(DT_EINVAL, "null context or output handle");
    *out = nullptr;
    dt_server *s = new dt_server();
    s->ctx = ctx;
    if (cfg) s->cfg = *cfg;
    if (!s->cfg.max_inflight_queries) s->cfg.max_inflight_queries = 4096;
    if (!s->cfg.max_batch) s->cfg.max_batch = 512;
    s->budget = s->cfg.hbm_budget_bytes ? s->cfg.hbm_budget_bytes : ctx->budget;
    (void)hipSetDevice(ctx->device);
    for (Slot &sl : s->slots) {
        int rc = make_batch_runner(ctx, &sl.runner);
        if (rc != DT_OK) {
            for (Slot &x : s->slots)
                if (x.runner) destroy_batch_runner(x.runner);
            delete s;
            return rc;
        }
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return DT_OK;
}

int dt_server_add_graph(dt_server *s, dt_graph *g, uint32_t *graph_id) {
    clear_error();
    if (!s || !g || !graph_id) return fail(DT_EINVAL, "null argument");
    if (g->ctx != s->ctx) return fail(DT_EINVAL, "graph belongs to another context");
    if (!g->built) return fail(DT_ENOTBUILT, "graph not built");
    const uint64_t bytes = graph_device_bytes(g);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->budget && s->used + bytes > s->budget)
        return fail(DT_ENOMEM, "graph needs %llu bytes; %llu of the server's %llu are in use",
                    (unsigned long long)bytes, (unsigned long long)s->used, (unsigned long long)s->budget);
    s->used += bytes;
    s->graphs.push_back(g);
    *graph_id = (uint32_t)(s->graphs.size() - 1);
    return DT_OK;
}

int dt_server_submit(dt_server *s, uint32_t graph_id, const dt_query *q, uint64_t *ticket) {
    clear_error();
    if (!s || !q || !ticket) return fail(DT_EINVAL, "null argument");
    dt_graph *g = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (graph_id >= s->graphs.size()) return fail(DT_EINVAL, "unknown graph id %u", graph_id);
        g = s->graphs[graph_id];
    }
    Ticket t;
    DT_TRY(normalise_query(g, q, &t.q, &t.empty));
    if ((g->sum_sigma3 >> 63) != 0) return fail(DT_EOVERFLOW, "counts of this graph may not fit int64");
    t.empty = t.empty || g->n_tri == 0;
    t.gid = graph_id;
    t.submitted = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(DT_EBUSY, "server is stopping");
    if (s->inflight >= s->cfg.max_inflight_queries)
        return fail(DT_EBUSY, "%u queries in flight (limit %u)", s->inflight, s->cfg.max_inflight_queries);
    const uint64_t id = s->next_ticket++;
    s->tickets.emplace(id, t);
    s->pending.push_back(id);
    s->inflight++;
    *ticket = id;
    s->cv_work.notify_one();
    return DT_OK;
}

int dt_server_wait(dt_server *s, uint64_t ticket, int64_t out[8], int64_t timeout_ns) {
    clear_error();
    if (!s || !out) return fail(DT_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(DT_EINVAL, "unknown or already collected ticket %llu", (unsigned long long)ticket);
    auto ready = [&] { return s->tickets[ticket].done; };
    if (timeout_ns < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready)) {
        return fail(DT_ETIMEDOUT, "ticket %llu not done within the timeout", (unsigned long long)ticket);
    }
    Ticket &t = s->tickets[ticket];
    for (int j = 0; j < 8; ++j) out[j] = t.out[j];
    const int rc = t.rc;
    s->tickets.erase(ticket);
    if (rc != DT_OK) return fail(rc, "query failed: %s", dt_strerror(rc));
    return DT_OK;
}

int dt_server_stop(dt_server *s) {
    clear_error();
    if (!s) return fail(DT_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (Slot &sl : s->slots)
        if (sl.runner) destroy_batch_runner(sl.runner);
    delete s;
    return DT_OK;
}

}  // extern "C"
