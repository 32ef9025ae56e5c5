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
//
// With host swapping, more graphs may be admitted than the budget holds: a graph that does not fit
// waits in host memory, and when a query needs it the worker moves the least recently used
// resident graphs that no batch on the device is using out to host memory until it fits, then
// copies it back in (a query whose graph cannot be brought in yet waits for batches to finish).
#include <chrono>
#include <unordered_map>

#include "internal.h"

namespace dt {

namespace {

// every device array of a graph, in a fixed order (the order of its host copies while swapped)
std::vector<DevMem *> graph_arrays(dt_graph *g) {
    return {&g->sx, &g->sy, &g->row, &g->col, &g->ceid, &g->psid, &g->pdir, &g->pkey,
            &g->pstart, &g->c1, &g->core, &g->rank, &g->order, &g->dag_row, &g->dag_col,
            &g->eoff, &g->key, &g->sched.light, &g->sched.medium, &g->sched.mitems,
            &g->sched.light_w, &g->sched.medium_w, &g->sched.mitems_w, &g->sched.heavy,
            &g->sched.hslot, &g->sched.chunks, &g->sched.pchunks, &g->sched.mlev_w,
            &g->sched.unit};
}

}  // namespace

uint64_t graph_device_bytes(const dt_graph *g) {
    uint64_t b = 0;
    if (g->swapped) {
        for (size_t x : g->swap_bytes) b += x;
    } else {
        for (const DevMem *m : graph_arrays(const_cast<dt_graph *>(g))) b += m->bytes;
    }
    // scratch of the heavy path, taken per query in flight
    b += g->sched.n_slots * 8 * sizeof(int64_t) + g->sched.n_pchunks * 8 * sizeof(int64_t) + 48 * g->sched.n_heavy;
    return b;
}

int graph_swap_out(dt_graph *g, hipStream_t st) {
    if (g->swapped) return DT_OK;
    std::vector<DevMem *> arrs = graph_arrays(g);
    std::vector<std::unique_ptr<uint8_t[]>> host(arrs.size());
    std::vector<size_t> bytes(arrs.size(), 0);
    for (size_t i = 0; i < arrs.size(); ++i) {
        if (!arrs[i]->ptr) continue;
        bytes[i] = arrs[i]->bytes;
        host[i].reset(new (std::nothrow) uint8_t[bytes[i]]);
        if (!host[i]) return fail(DT_ENOMEM, "no host memory for %zu bytes of a swapped graph", bytes[i]);
        DT_HIP(hipMemcpyAsync(host[i].get(), arrs[i]->ptr, bytes[i], hipMemcpyDeviceToHost, st));
    }
    DT_HIP(hipStreamSynchronize(st));
    for (DevMem *m : arrs) m->reset();
    g->swap_host = std::move(host);
    g->swap_bytes = std::move(bytes);
    g->swapped = true;
    return DT_OK;
}

int graph_swap_in(dt_graph *g, hipStream_t st) {
    if (!g->swapped) return DT_OK;
    std::vector<DevMem *> arrs = graph_arrays(g);
    int rc = DT_OK;
    for (size_t i = 0; i < arrs.size() && rc == DT_OK; ++i) {
        if (!g->swap_bytes[i]) continue;
        rc = dev_alloc(g->ctx, *arrs[i], g->swap_bytes[i], false);
        if (rc == DT_OK && hipMemcpyAsync(arrs[i]->ptr, g->swap_host[i].get(), g->swap_bytes[i],
                                          hipMemcpyHostToDevice, st) != hipSuccess)
            rc = fail(DT_EDEVICE, "copy of a swapped graph back to the device failed");
    }
    if (rc == DT_OK && hipStreamSynchronize(st) != hipSuccess)
        rc = fail(DT_EDEVICE, "copy of a swapped graph back to the device failed");
    if (rc != DT_OK) {
        // the host copies stay: the graph is still swapped out
        (void)hipStreamSynchronize(st);
        for (DevMem *m : arrs) m->reset();
        return rc;
    }
    g->swap_host.clear();
    g->swap_bytes.clear();
    g->swapped = false;
    return DT_OK;
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
    std::vector<uint32_t> gids;
    std::vector<dt_graph *> graphs;
    std::vector<DQuery> qs;
    std::unique_ptr<bool[]> empty;
    size_t cap = 0;
};

// an admitted graph: its device bytes (with the heavy path's scratch), whether its arrays are in
// HBM, the batches on the device that use it, and when a batch last took it
struct Served {
    dt_graph *g = nullptr;
    uint64_t bytes = 0;
    bool resident = true;
    uint32_t users = 0;
    uint64_t last_use = 0;
};

constexpr int kNoRoom = 1;   // make_resident: every graph that could move out is in use

}  // namespace
}  // namespace dt

struct dt_server {
    dt_ctx *ctx = nullptr;
    dt_server_cfg cfg{};
    uint64_t budget = 0, used = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<dt::Served> graphs;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, dt::Ticket> tickets;
    uint64_t next_ticket = 1;
    uint32_t inflight = 0;
    bool stopping = false;
    int worker_rc = DT_OK;
    dt::Slot slots[dt::kSlots];
    std::thread worker;
    hipStream_t copy = nullptr;   // the worker's swap copies
    uint64_t clock = 0, swap_outs = 0, swap_ins = 0, swap_out_bytes = 0, swap_in_bytes = 0, done = 0;
};

namespace dt {
namespace {

// the slot's graphs are no longer used by a batch on the device (lock held)
void release_graphs(dt_server *s, Slot &sl) {
    for (uint32_t gid : sl.gids) s->graphs[gid].users--;
    sl.gids.clear();
}

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
    s->done += k;
    release_graphs(s, sl);
    sl.busy = false;
    sl.tickets.clear();
    s->cv_done.notify_all();
}

// Brings graph gid into HBM, first moving least recently used resident graphs that no batch uses
// out to host memory until it fits the budget.  Called by the worker with the lock held; releases
// it during copies (only the worker moves graphs, and the graphs it moves are in no batch).
// Returns DT_OK, kNoRoom (every graph that could move out is in use: wait for batches), or an error.
int make_resident(dt_server *s, std::unique_lock<std::mutex> &lk, uint32_t gid) {
    const uint64_t need = s->graphs[gid].bytes;
    while (s->budget && s->used + need > s->budget) {
        int victim = -1;
        for (size_t i = 0; i < s->graphs.size(); ++i) {
            const Served &e = s->graphs[i];
            if (i == gid || !e.resident || e.users) continue;
            if (victim < 0 || e.last_use < s->graphs[victim].last_use) victim = (int)i;
        }
        if (victim < 0) return kNoRoom;
        dt_graph *vg = s->graphs[victim].g;
        const uint64_t vb = s->graphs[victim].bytes;
        s->graphs[victim].resident = false;
        s->used -= vb;
        lk.unlock();
        const int rc = graph_swap_out(vg, s->copy);
        lk.lock();
        if (rc != DT_OK) {
            s->graphs[victim].resident = true;
            s->used += vb;
            return rc;
        }
        s->swap_outs++;
        s->swap_out_bytes += vb;
    }
    dt_graph *g = s->graphs[gid].g;
    s->graphs[gid].resident = true;
    s->used += need;
    lk.unlock();
    const int rc = graph_swap_in(g, s->copy);
    lk.lock();
    if (rc != DT_OK) {
        s->graphs[gid].resident = false;
        s->used -= need;
        return rc;
    }
    s->swap_ins++;
    s->swap_in_bytes += need;
    return DT_OK;
}

void finish_ticket(dt_server *s, Ticket &t, int rc) {
    t.rc = rc;
    t.done = true;
    s->inflight--;
    s->done++;
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
            sl.gids.clear();
            sl.graphs.clear();
            sl.qs.clear();
            const auto now = std::chrono::steady_clock::now();
            while (!s->pending.empty() && sl.tickets.size() < max_batch) {
                const uint64_t id = s->pending.front();
                Ticket &t = s->tickets[id];   // (references into the map survive its rehashing)
                if (deadline > 0 &&
                    std::chrono::duration_cast<std::chrono::nanoseconds>(now - t.submitted).count() > deadline) {
                    s->pending.pop_front();
                    finish_ticket(s, t, fail(DT_ETIMEDOUT, "query passed its deadline before reaching the device"));
                    progressed = true;
                    continue;
                }
                const uint32_t gid = t.gid;
                if (!s->graphs[gid].resident) {
                    const int rc = make_resident(s, lk, gid);
                    if (rc == kNoRoom) break;   // run what is taken; the rest waits for room
                    if (rc != DT_OK) {
                        s->pending.pop_front();
                        finish_ticket(s, t, rc);
                        progressed = true;
                        continue;
                    }
                }
                s->pending.pop_front();
                Served &e = s->graphs[gid];
                e.users++;
                e.last_use = ++s->clock;
                sl.tickets.push_back(id);
                sl.gids.push_back(gid);
                sl.graphs.push_back(e.g);
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
                    s->done += k;
                    release_graphs(s, sl);
                    sl.busy = false;
                    sl.tickets.clear();
                    s->cv_done.notify_all();
                }
                progressed = true;
            }
        }
        bool any_busy = false;
        for (Slot &sl : s->slots) any_busy |= sl.busy;
        if (s->stopping && s->pending.empty() && !any_busy) break;
        if (progressed) continue;
        if (any_busy) {
            bool all_busy = true;
            for (Slot &sl : s->slots) all_busy &= sl.busy;
            if (all_busy || !s->pending.empty()) {
                // nothing can start until a batch ends (no runner free, or the waiting queries'
                // graphs need room that batches on the device hold): wait for the oldest
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
    if (cfg && cfg->swap_to_host > 1) return fail(DT_EINVAL, "swap_to_host is 0 or 1");
    dt_server *s = new dt_server();
    s->ctx = ctx;
    if (cfg) s->cfg = *cfg;
    if (!s->cfg.max_inflight_queries) s->cfg.max_inflight_queries = 4096;
    if (!s->cfg.max_batch) s->cfg.max_batch = 512;
    s->budget = s->cfg.hbm_budget_bytes ? s->cfg.hbm_budget_bytes : ctx->budget;
    (void)hipSetDevice(ctx->device);
    int rc = DT_OK;
    if (hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess)
        rc = fail(DT_EDEVICE, "hipStreamCreateWithFlags failed");
    for (Slot &sl : s->slots)
        if (rc == DT_OK) rc = make_batch_runner(ctx, &sl.runner);
    if (rc != DT_OK) {
        for (Slot &x : s->slots)
            if (x.runner) destroy_batch_runner(x.runner);
        if (s->copy) (void)hipStreamDestroy(s->copy);
        delete s;
        return rc;
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return DT_OK;
}

int dt_server_add_graph(dt_server *s, dt_graph *g, uint32_t *graph_id) {
    clear_error();
    if (!s || !g || !graph_id) return fail(DT_EINVAL, "null argument");
    if (g->ctx != s->ctx) return fail(DT_EINVAL, "graph belongs to another context");
    if (g->held_by) return fail(DT_EBUSY, "graph is already held by a server that swaps graphs");
    DT_TRY(check_graph(g, true));   // (a graph a stopped server left in host memory comes back)
    const uint64_t bytes = graph_device_bytes(g);
    const bool swap = s->cfg.swap_to_host != 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (swap)
        for (const Served &e : s->graphs)
            if (e.g == g) return fail(DT_EINVAL, "graph already admitted");
    const bool fits = !s->budget || s->used + bytes <= s->budget;
    if (!fits && (!swap || bytes > s->budget))
        return fail(DT_ENOMEM, "graph needs %llu bytes; %llu of the server's %llu are in use",
                    (unsigned long long)bytes, (unsigned long long)s->used, (unsigned long long)s->budget);
    Served e;
    e.g = g;
    e.bytes = bytes;
    e.resident = fits;
    if (!fits) {
        // the graph waits in host memory until a query needs it (it is in no batch yet, and the
        // caller's work on it is finished once the context's stream is)
        lk.unlock();
        DeviceGuard dg(s->ctx->device);
        DT_TRY(relayout_join(g));
        DT_HIP(hipStreamSynchronize(s->ctx->stream));
        DT_TRY(graph_swap_out(g, s->ctx->stream));
        lk.lock();
        s->swap_outs++;
        s->swap_out_bytes += bytes;
    } else {
        s->used += bytes;
    }
    if (swap) g->held_by = s;
    s->graphs.push_back(e);
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
        g = s->graphs[graph_id].g;
    }
    Ticket t;
    DT_TRY(normalise_query(g, q, &t.q, &t.empty));   // (host fields only)
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

int dt_server_stats(dt_server *s, dt_server_info *out) {
    clear_error();
    if (!s || !out) return fail(DT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    dt_server_info r{};
    r.graphs = s->graphs.size();
    for (const Served &e : s->graphs) r.resident_graphs += e.resident ? 1 : 0;
    r.resident_bytes = s->used;
    r.budget_bytes = s->budget;
    r.swap_outs = s->swap_outs;
    r.swap_ins = s->swap_ins;
    r.swap_out_bytes = s->swap_out_bytes;
    r.swap_in_bytes = s->swap_in_bytes;
    r.queries_done = s->done;
    *out = r;
    return DT_OK;
}

int dt_server_graph_info(dt_server *s, uint32_t graph_id, int *resident, uint64_t *bytes) {
    clear_error();
    if (!s || !resident || !bytes) return fail(DT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id >= s->graphs.size()) return fail(DT_EINVAL, "unknown graph id %u", graph_id);
    *resident = s->graphs[graph_id].resident ? 1 : 0;
    *bytes = s->graphs[graph_id].bytes;
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
    // the graphs go back to the caller; one left in host memory returns to HBM on its next use
    for (Served &e : s->graphs)
        if (e.g->held_by == s) e.g->held_by = nullptr;
    if (s->copy) (void)hipStreamDestroy(s->copy);
    delete s;
    return DT_OK;
}

}  // extern "C"
