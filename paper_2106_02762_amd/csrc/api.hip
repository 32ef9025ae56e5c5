// The C ABI (include/dottt.h): contexts, graph load / build / statistics, counts.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace dt {
const char *last_error();

namespace {

constexpr unsigned kBlock = 256;

// node ids (a < b < c) of every resident triangle
__global__ void k_tri_vertices(uint64_t nt, const uint32_t *__restrict__ tri, uint32_t n,
                               const uint32_t *__restrict__ dag_row, const uint32_t *__restrict__ dag_col,
                               const uint32_t *__restrict__ order, uint32_t *__restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nt) return;
    const uint32_t e_uv = tri[3 * i], e_uw = tri[3 * i + 1];
    if (e_uv == kNoEdge) {   // an empty list entry stays empty
        out[3 * i] = out[3 * i + 1] = out[3 * i + 2] = kNoEdge;
        return;
    }
    // tail of e_uv: the last u with dag_row[u] <= e_uv
    uint32_t lo = 0, len = n;
    while (len > 0) {
        uint32_t half = len >> 1;
        if (dag_row[lo + half + 1] <= e_uv) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    uint32_t a = order[lo], b = order[dag_col[e_uv]], c = order[dag_col[e_uw]];
    uint32_t x = min(a, min(b, c)), z = max(a, max(b, c));
    uint32_t y = a ^ b ^ c ^ x ^ z;
    out[3 * i] = x;
    out[3 * i + 1] = y;
    out[3 * i + 2] = z;
}

// The split and geometry of the next schedule: the user's fields where set, else the autotuner's
// choice for g's size class (tuning it first when allowed and not cached: graphs of at least 2^20
// static triangles, both split fields automatic, no forced path), else the defaults.
int resolve_split(dt_graph *g, DevMem *tri) {
    const dt_tuning &tu = g->tuning;
    TunedCount t;
    bool have = tu.autotune != 1 && tuned_lookup(g, &t);
    const bool auto_split = tu.light_pair_cap == 0 && tu.medium_cost_pct == 0 && tu.force_path == 0;
    g->tuned = 0;
    if (tri && auto_split && tu.autotune != 1 && (tu.autotune == 2 || (!have && g->n_tri >= (1ull << 20)))) {
        DT_TRY(autotune_count(g, *tri, &t));
        have = true;
        if (g->tuning.autotune == 2) g->tuning.autotune = 0;
    }
    if (!have || !auto_split) t = TunedCount();
    g->light_cap_used = tu.light_pair_cap ? tu.light_pair_cap : t.light_cap;
    g->cost_pct_used = tu.medium_cost_pct ? tu.medium_cost_pct : t.cost_pct;
    g->geom.light_bpc = t.light_bpc;
    g->geom.medium_bpc = t.medium_bpc;
    g->tuned = have && auto_split ? 1 : 0;
    return DT_OK;
}


int load_common(dt_ctx *ctx, uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst,
                const int64_t *t, bool on_device, dt_graph **out) {
    if (!ctx || !out) return fail(DT_EINVAL, "null context or output handle");
    *out = nullptr;
    if (m && (!src || !dst || !t)) return fail(DT_EINVAL, "null edge array");
    if (m >= (1ull << 31)) return fail(DT_EOVERFLOW, "m = %llu edges; this version takes m < 2^31",
                                       (unsigned long long)m);
    if (n >= (1u << 31)) return fail(DT_EOVERFLOW, "n = %u vertices; this version takes n < 2^31", n);
    DeviceGuard dg(ctx->device);
    double t0 = now_ms();
    dt_graph *g = new dt_graph();
    g->ctx = ctx;
    g->n = n;
    g->m_in = m;
    int rc = DT_OK;
    if (on_device || m == 0) {
        rc = load_graph(g, src, dst, t);
    } else {
        DevMem ds, dd, dtm;
        rc = dev_alloc(ctx, ds, m * 4);
        if (rc == DT_OK) rc = dev_alloc(ctx, dd, m * 4);
        if (rc == DT_OK) rc = dev_alloc(ctx, dtm, m * 8);
        if (rc == DT_OK) {
            hipError_t e = hipMemcpy(ds.ptr, src, m * 4, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(dd.ptr, dst, m * 4, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(dtm.ptr, t, m * 8, hipMemcpyHostToDevice);
            if (e != hipSuccess) rc = fail(DT_EDEVICE, "copy of the edge arrays failed: %s", hipGetErrorString(e));
        }
        if (rc == DT_OK) rc = load_graph(g, ds.as<uint32_t>(), dd.as<uint32_t>(), dtm.as<int64_t>());
    }
    if (rc != DT_OK) {
        delete g;
        return rc;
    }
    g->ms_load = now_ms() - t0;
    *out = g;
    return DT_OK;
}

}  // namespace

int check_graph(const dt_graph *g, bool need_built, bool device) {
    if (!g) return fail(DT_EINVAL, "null graph");
    if (need_built && !g->built) return fail(DT_ENOTBUILT, "graph not built (call dt_graph_build)");
    if (device && g->held_by)
        return fail(DT_EBUSY, "the graph is held by a server that swaps graphs to host memory; "
                              "count it through the server until dt_server_stop");
    if (device && g->swapped) {
        dt_graph *w = const_cast<dt_graph *>(g);   // the arrays come back unchanged
        DeviceGuard dg(w->ctx->device);
        DT_TRY(graph_swap_in(w, w->ctx->stream));
    }
    return DT_OK;
}

}  // namespace dt

using namespace dt;

extern "C" {

const char *dt_strerror(int code) {
    switch (code) {
        case DT_OK: return "ok";
        case DT_EINVAL: return "invalid argument";
        case DT_ENOMEM: return "out of device memory or over the HBM budget";
        case DT_EOVERFLOW: return "size limit exceeded or count may overflow int64";
        case DT_EBUSY: return "busy";
        case DT_ETIMEDOUT: return "timed out";
        case DT_EDEVICE: return "HIP runtime error";
        case DT_ENOTBUILT: return "graph not built";
        default: return "unknown error";
    }
}

const char *dt_last_error(void) { return dt::last_error(); }

int dt_ctx_create(int hip_device, uint64_t hbm_budget_bytes, dt_ctx **out) {
    clear_error();
    if (!out) return fail(DT_EINVAL, "null output handle");
    *out = nullptr;
    int ndev = 0;
    DT_HIP(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev)
        return fail(DT_EINVAL, "device %d not present (%d devices)", hip_device, ndev);
    DeviceGuard dg(hip_device);
    dt_ctx *c = new dt_ctx();
    c->device = hip_device;
    c->budget = hbm_budget_bytes;
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, hip_device);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->pinned_out, 64 * sizeof(int64_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->pinned_stage, kPinnedStage, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_a, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_b, hipEventDisableTiming);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_relay[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    auto release = [](dt_ctx *x) {
        x->out8.reset();
        if (x->ev_a) (void)hipEventDestroy(x->ev_a);
        if (x->ev_b) (void)hipEventDestroy(x->ev_b);
        for (int i = 0; i < 2; ++i) {
            if (x->side[i]) (void)hipStreamDestroy(x->side[i]);
            if (x->ev_join[i]) (void)hipEventDestroy(x->ev_join[i]);
            if (x->ev_relay[i]) (void)hipEventDestroy(x->ev_relay[i]);
        }
        if (x->ev_fork) (void)hipEventDestroy(x->ev_fork);
        if (x->pinned_out) (void)hipHostFree(x->pinned_out);
        if (x->pinned_stage) (void)hipHostFree(x->pinned_stage);
        if (x->stream) (void)hipStreamDestroy(x->stream);
        delete x;
    };
    if (e != hipSuccess) {
        release(c);
        return fail(DT_EDEVICE, "context setup failed: %s", hipGetErrorString(e));
    }
    if (c->num_cus <= 0) c->num_cus = 256;
    // the no-allocation count's scratch address on this device (taken once per device)
    int rc = noalloc_init(hip_device);
    if (rc == DT_OK) rc = dev_alloc(c, c->out8, 64 * sizeof(int64_t), false);
    if (rc != DT_OK) {
        release(c);
        return rc;
    }
    *out = c;
    return DT_OK;
}

int dt_ctx_destroy(dt_ctx *ctx) {
    clear_error();
    if (!ctx) return fail(DT_EINVAL, "null context");
    DeviceGuard dg(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->batch) destroy_batch_runner(ctx->batch);
    ctx->batch = nullptr;
    ctx->scratch.partials.reset();
    ctx->scratch.heavy_vals.reset();
    ctx->scratch.sweep_partials.reset();
    ctx->out8.reset();
    pool_trim(ctx, 0);
    if (ctx->pinned_out) (void)hipHostFree(ctx->pinned_out);
    if (ctx->pinned_stage) (void)hipHostFree(ctx->pinned_stage);
    for (auto &e : ctx->prof_ev)
        if (e) (void)hipEventDestroy(e);
    for (int i = 0; i < 2; ++i) {
        if (ctx->side[i]) (void)hipStreamSynchronize(ctx->side[i]);
        if (ctx->side[i]) (void)hipStreamDestroy(ctx->side[i]);
        if (ctx->ev_join[i]) (void)hipEventDestroy(ctx->ev_join[i]);
        if (ctx->ev_relay[i]) (void)hipEventDestroy(ctx->ev_relay[i]);
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    (void)hipEventDestroy(ctx->ev_a);
    (void)hipEventDestroy(ctx->ev_b);
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return DT_OK;
}

int dt_ctx_memory(const dt_ctx *ctx, uint64_t *used, uint64_t *budget) {
    clear_error();
    if (!ctx) return fail(DT_EINVAL, "null context");
    if (used) *used = ctx->used.load();
    if (budget) *budget = ctx->budget;
    return DT_OK;
}

int dt_graph_load(dt_ctx *ctx, uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst,
                  const int64_t *t, dt_graph **out) {
    clear_error();
    return load_common(ctx, n, m, src, dst, t, false, out);
}

int dt_graph_load_device(dt_ctx *ctx, uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst,
                         const int64_t *t, dt_graph **out) {
    clear_error();
    return load_common(ctx, n, m, src, dst, t, true, out);
}

int dt_graph_build(dt_graph *g) {
    clear_error();
    DT_TRY(check_graph(g, false));
    DeviceGuard dg(g->ctx->device);
    prof_clear(g->ctx, true);
    g->built = false;
    double t0 = now_ms();
    DT_TRY(order_vertices(g));
    double t1 = now_ms();
    DT_TRY(orient(g, true));
    double t2 = now_ms();
    DevMem tri;
    uint64_t ntri = 0, cand = 0, nlist = 0;
    {
        // the store's re-layout runs beside the enumeration, which does not read it
        struct Join {
            dt_graph *g;
            ~Join() { (void)relayout_join(g); }
        } join{g};
        DT_TRY(enumerate_triangles(g, tri, &ntri, &cand, &nlist));
        DT_TRY(relayout_join(g));
    }
    g->n_tri = ntri;
    g->n_tri_list = nlist;
    g->tri_candidates = cand;
    g->alg_bytes_tri = 4 * (g->m_s + cand) + 12 * ntri;
    double t3 = now_ms();
    DT_TRY(resolve_split(g, &tri));
    DT_TRY(make_schedule(g, tri));
    double t4 = now_ms();
    g->ms_peel = t1 - t0;
    g->ms_orient = t2 - t1;
    g->ms_tri = t3 - t2;
    g->ms_sched = t4 - t3;
    g->built = true;
    return DT_OK;
}

int dt_graph_set_tuning(dt_graph *g, const dt_tuning *tu) {
    clear_error();
    DT_TRY(check_graph(g, false));
    if (!tu) return fail(DT_EINVAL, "null tuning");
    dt_tuning nt = g->tuning;
    if (tu->light_pair_cap) nt.light_pair_cap = tu->light_pair_cap;
    if (tu->medium_cost_pct) nt.medium_cost_pct = tu->medium_cost_pct;
    if (tu->autotune > 2) return fail(DT_EINVAL, "autotune must be 0, 1 or 2");
    nt.autotune = tu->autotune;
    if (tu->heavy_chunk) nt.heavy_chunk = tu->heavy_chunk;
    if (tu->medium_pair_cap) nt.medium_pair_cap = tu->medium_pair_cap;
    if (tu->force_path > 3) return fail(DT_EINVAL, "force_path must be 0, 1, 2 or 3");
    nt.force_path = tu->force_path;
    if (tu->peel_tail > kPeelTailMax) return fail(DT_EINVAL, "peel_tail must be at most %u", kPeelTailMax);
    if (tu->peel_tail) nt.peel_tail = tu->peel_tail;
    if (tu->order_method > 1) return fail(DT_EINVAL, "order_method must be 0 or 1");
    nt.order_method = tu->order_method;
    if (nt.heavy_chunk != 256) return fail(DT_EINVAL, "heavy_chunk must be 256 in this version");
    if (nt.medium_pair_cap > (1u << 30)) return fail(DT_EINVAL, "medium_pair_cap must be at most 2^30");
    g->tuning = nt;
    if (!g->built) return DT_OK;
    // re-split the triangles under the new tuning (unit triangles keep no edge ids, so the
    // enumeration pass runs again; it yields the same triangles)
    DeviceGuard dg(g->ctx->device);
    DevMem tri;
    uint64_t ntri = 0, cand = 0, nlist = 0;
    DT_TRY(enumerate_triangles(g, tri, &ntri, &cand, &nlist));
    if (ntri != g->n_tri) return fail(DT_EDEVICE, "triangle enumeration changed between passes");
    g->n_tri_list = nlist;
    DT_TRY(resolve_split(g, g->tuning.autotune == 2 ? &tri : nullptr));
    return make_schedule(g, tri);
}

int dt_graph_stats(const dt_graph *g, dt_stats *out) {
    clear_error();
    DT_TRY(check_graph(g, false, false));
    if (!out) return fail(DT_EINVAL, "null output");
    memset(out, 0, sizeof(*out));
    out->n = g->n;
    out->m = g->m_in;
    out->m_loaded = g->m;
    out->self_loops_dropped = g->self_loops;
    out->m_static = g->m_s;
    out->max_multiplicity = g->max_mult;
    out->t_min = g->m ? g->t_min : INT64_MAX;
    out->t_max = g->m ? g->t_max : INT64_MIN;
    out->ms_load = g->ms_load;
    if (g->built) {
        out->n_static_triangles = g->n_tri;
        out->degeneracy = g->kappa;
        out->max_out_degree = g->max_outdeg;
        out->peel_rounds = g->peel_rounds;
        out->sum_sigma3_lo = (uint64_t)g->sum_sigma3;
        out->sum_sigma3_hi = (uint64_t)(g->sum_sigma3 >> 64);
        out->n_light_triangles = g->sched.n_light;
        out->n_heavy_triangles = g->sched.n_heavy;
        out->n_medium_triangles = g->sched.n_medium;
        out->n_unit_triangles = g->sched.n_unit;
        out->alg_bytes = g->alg_bytes;
        out->alg_bytes_light = g->alg_bytes_light;
        out->alg_bytes_medium = g->alg_bytes_medium;
        out->alg_bytes_unit = g->alg_bytes_unit;
        out->alg_bytes_peel = g->alg_bytes_peel;
        out->alg_bytes_triangles = g->alg_bytes_tri;
        out->tri_candidates = g->tri_candidates;
        out->heavy_slots = g->sched.n_slots;
        out->ms_peel = g->ms_peel;
        out->ms_orient = g->ms_orient;
        out->ms_triangles = g->ms_tri;
        out->ms_schedule = g->ms_sched;
        out->n_contested_triangles = g->sched.n_contested;
        out->light_pair_cap_used = g->light_cap_used;
        out->medium_cost_pct_used = g->cost_pct_used;
        out->light_blocks_per_cu = g->geom.light_bpc;
        out->medium_blocks_per_cu = g->geom.medium_bpc;
        out->autotuned = (uint32_t)g->tuned;
    }
    return DT_OK;
}

// Checks the graph and normalises the query.  A graph whose sum of multiplicity products reaches
// 2^63 may have counts beyond int64: only the calls that count in 128 bits (allow_wide) take it.
static int count_guarded(dt_graph *g, const dt_query *q, DQuery *dq, bool *empty, bool allow_wide = false) {
    DT_TRY(check_graph(g, true));
    DT_TRY(normalise_query(g, q, dq, empty));
    if (!allow_wide && (g->sum_sigma3 >> 63) != 0)
        return fail(DT_EOVERFLOW, "the sum of multiplicity products exceeds 2^63; counts may not fit int64 "
                                  "(dt_count and dt_count_visits count such graphs in 128 bits)");
    return DT_OK;
}

// The 128-bit result of a wide count, (low, high) word pairs per type, into int64 counts; a type
// whose count reaches 2^63 is refused and out is left as it was.
static int narrow_counts(const int64_t *w16, const int64_t *add8, int64_t out[8]) {
    int64_t r[8];
    for (int i = 0; i < 8; ++i) {
        unsigned __int128 v = ((unsigned __int128)(uint64_t)w16[2 * i + 1] << 64) | (uint64_t)w16[2 * i];
        if (add8) v += (uint64_t)add8[i];
        if ((v >> 63) != 0) return fail(DT_EOVERFLOW, "the count of type T%d reaches 2^63", i + 1);
        r[i] = (int64_t)(uint64_t)v;
    }
    memcpy(out, r, sizeof(r));
    return DT_OK;
}

int dt_count(dt_graph *g, const dt_query *q, int64_t out[8]) {
    clear_error();
    if (!out) return fail(DT_EINVAL, "null output");
    DQuery dq;
    bool empty = false;
    DT_TRY(count_guarded(g, q, &dq, &empty, true));
    if (empty || g->n_tri == 0) {
        for (int i = 0; i < 8; ++i) out[i] = 0;
        return DT_OK;
    }
    dt_ctx *ctx = g->ctx;
    DeviceGuard dg(ctx->device);
    const bool wide = (g->sum_sigma3 >> 63) != 0;
    const size_t words = wide ? 16 : 8;
    DT_TRY(count_enqueue(g, dq, ctx->out8.as<int64_t>(), ctx->stream, false, nullptr, ctx->scratch));
    DT_HIP(hipMemcpyAsync(ctx->pinned_out, ctx->out8.ptr, words * sizeof(int64_t), hipMemcpyDeviceToHost,
                          ctx->stream));
    DT_HIP(hipStreamSynchronize(ctx->stream));
    if (wide) return narrow_counts(ctx->pinned_out, nullptr, out);
    memcpy(out, ctx->pinned_out, 8 * sizeof(int64_t));
    return DT_OK;
}

int dt_count_oneshot(dt_graph *g, const dt_query *q, int64_t out[8]) {
    clear_error();
    DT_TRY(check_graph(g, false));
    if (!out) return fail(DT_EINVAL, "null output");
    DQuery dq;
    bool empty = false;
    DT_TRY(normalise_query(g, q, &dq, &empty));
    for (int i = 0; i < 8; ++i) out[i] = 0;
    if (empty) return DT_OK;
    dt_ctx *ctx = g->ctx;
    DeviceGuard dg(ctx->device);
    // the split of the last build (or the user's, or the defaults)
    if (g->tuning.light_pair_cap) g->light_cap_used = g->tuning.light_pair_cap;
    if (!g->light_cap_used) g->light_cap_used = 4;
    if (g->tuning.medium_cost_pct) g->cost_pct_used = g->tuning.medium_cost_pct;
    if (!g->cost_pct_used) g->cost_pct_used = 100;
    // the cached products of an earlier build refer to the ordering about to be replaced
    g->built = false;
    g->sched = Schedule();
    g->n_tri = 0;
    double t0 = now_ms();
    DT_TRY(order_vertices(g));
    double t1 = now_ms();
    DT_TRY(orient(g));
    double t2 = now_ms();
    int64_t *o = ctx->out8.as<int64_t>();
    DevMem rest;
    uint64_t n_rest = 0, ntri = 0, cand = 0;
    DT_TRY(fused_count(g, dq, o, rest, &n_rest, &ntri, &cand));
    g->tri_candidates = cand;
    const unsigned __int128 s3_all = g->sum_sigma3;   // of every triangle (the schedule's is the rest's)
    int rc = DT_OK;
    // the light triangles are summed in int64: each adds at most light_pair_cap * 64 triples
    if (((unsigned __int128)ntri * g->light_cap_used * 64) >> 63)
        rc = fail(DT_EOVERFLOW, "the one-pass count's int64 sums of %llu light triangles may overflow; "
                                "build the graph and count with dt_count", (unsigned long long)ntri);
    if (rc == DT_OK && n_rest) {
        // the triangles for the medium and heavy paths: a schedule of their own, then a count
        // (the rest is counted in 128 bits when its sum of multiplicity products reaches 2^63, 16
        // words at o + 8)
        g->n_tri = n_rest;
        g->n_tri_list = n_rest;
        rc = make_schedule(g, rest);
        if (rc == DT_OK) rc = count_enqueue(g, dq, o + 8, ctx->stream, false, nullptr, ctx->scratch);
    } else if (rc == DT_OK) {
        DT_HIP(hipMemsetAsync(o + 8, 0, 8 * sizeof(int64_t), ctx->stream));
    }
    if (rc == DT_OK) {
        const bool wide = n_rest && (g->sum_sigma3 >> 63) != 0;
        DT_HIP(hipMemcpyAsync(ctx->pinned_out, o, (wide ? 24 : 16) * sizeof(int64_t), hipMemcpyDeviceToHost,
                              ctx->stream));
        DT_HIP(hipStreamSynchronize(ctx->stream));
        if (wide) {
            rc = narrow_counts(ctx->pinned_out + 8, ctx->pinned_out, out);
        } else {
            for (int i = 0; i < 8; ++i) out[i] = ctx->pinned_out[i] + ctx->pinned_out[8 + i];
        }
    }
    g->sched = Schedule();
    g->n_tri = ntri;
    g->sum_sigma3 = s3_all;
    g->ms_peel = t1 - t0;
    g->ms_orient = t2 - t1;
    g->ms_tri = now_ms() - t2;
    g->ms_sched = 0;
    return rc;
}

int dt_count_sweep(dt_graph *g, uint64_t k, const dt_query *queries, int64_t *out) {
    clear_error();
    if (!queries || !out) return fail(DT_EINVAL, "null queries or output");
    for (uint64_t j = 1; j < k; ++j)
        if (queries[j].t_lo != queries[0].t_lo || queries[j].t_hi != queries[0].t_hi)
            return fail(DT_EINVAL, "the queries of a sweep share one window (query %llu differs)",
                        (unsigned long long)j);
    for (uint64_t b = 0; b < k; b += kSweepMax) {
        const uint32_t kk = (uint32_t)std::min<uint64_t>(kSweepMax, k - b);
        DQuery dq[kSweepMax];
        bool empty = false;
        for (uint32_t j = 0; j < kk; ++j) DT_TRY(count_guarded(g, &queries[b + j], &dq[j], &empty));
        if (empty || g->n_tri == 0) {
            for (uint64_t i = 0; i < 8ull * kk; ++i) out[8 * b + i] = 0;
            continue;
        }
        dt_ctx *ctx = g->ctx;
        DeviceGuard dg(ctx->device);
        DT_TRY(count_sweep_enqueue(g, dq, kk, ctx->out8.as<int64_t>(), ctx->stream, ctx->scratch));
        DT_HIP(hipMemcpyAsync(ctx->pinned_out, ctx->out8.ptr, 8 * kk * sizeof(int64_t), hipMemcpyDeviceToHost,
                              ctx->stream));
        DT_HIP(hipStreamSynchronize(ctx->stream));
        memcpy(out + 8 * b, ctx->pinned_out, 8 * kk * sizeof(int64_t));
    }
    return DT_OK;
}

int dt_count_async(dt_graph *g, const dt_query *q, int64_t *out8, void *hip_stream) {
    clear_error();
    if (!out8) return fail(DT_EINVAL, "null output");
    DQuery dq;
    bool empty = false;
    DT_TRY(count_guarded(g, q, &dq, &empty));
    dt_ctx *ctx = g->ctx;
    DeviceGuard dg(ctx->device);
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    if (empty || g->n_tri == 0) {
        DT_HIP(hipMemsetAsync(out8, 0, 8 * sizeof(int64_t), s));
        return DT_OK;
    }
    // the scratch (partials, heavy prefixes) belongs to the context: a foreign stream waits for
    // the context's stream before the count and the context's stream waits for it afterwards
    if (s != ctx->stream) {
        DT_HIP(hipEventRecord(ctx->ev_a, ctx->stream));
        DT_HIP(hipStreamWaitEvent(s, ctx->ev_a, 0));
    }
    DT_TRY(count_enqueue(g, dq, out8, s, false, nullptr, ctx->scratch));
    if (s != ctx->stream) {
        DT_HIP(hipEventRecord(ctx->ev_b, s));
        DT_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_b, 0));
    }
    return DT_OK;
}

int dt_count_visits(dt_graph *g, const dt_query *q, int64_t out[8], uint64_t *visits) {
    clear_error();
    if (!out || !visits) return fail(DT_EINVAL, "null output");
    DQuery dq;
    bool empty = false;
    DT_TRY(count_guarded(g, q, &dq, &empty, true));
    *visits = 0;
    if (empty || g->n_tri == 0) {
        for (int i = 0; i < 8; ++i) out[i] = 0;
        return DT_OK;
    }
    dt_ctx *ctx = g->ctx;
    DeviceGuard dg(ctx->device);
    // the counts in out8[0..8) (or [0..16) in 128 bits), the visits in out8[16]
    const bool wide = (g->sum_sigma3 >> 63) != 0;
    int64_t *o = ctx->out8.as<int64_t>();
    unsigned long long *v = reinterpret_cast<unsigned long long *>(o + 16);
    DT_HIP(hipMemsetAsync(v, 0, 8, ctx->stream));
    DT_TRY(count_enqueue(g, dq, o, ctx->stream, false, nullptr, ctx->scratch, 15, v));
    DT_HIP(hipMemcpyAsync(ctx->pinned_out, o, 17 * sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    DT_HIP(hipStreamSynchronize(ctx->stream));
    *visits = (uint64_t)ctx->pinned_out[16];
    if (wide) return narrow_counts(ctx->pinned_out, nullptr, out);
    memcpy(out, ctx->pinned_out, 8 * sizeof(int64_t));
    return DT_OK;
}

int dt_count_cells(dt_graph *g, const dt_query *q, int64_t out[48]) {
    clear_error();
    if (!out) return fail(DT_EINVAL, "null output");
    DQuery dq;
    bool empty = false;
    DT_TRY(count_guarded(g, q, &dq, &empty));
    if (empty || g->n_tri == 0) {
        for (int i = 0; i < 48; ++i) out[i] = 0;
        return DT_OK;
    }
    dt_ctx *ctx = g->ctx;
    DeviceGuard dg(ctx->device);
    DevMem cells;
    DT_TRY(dev_alloc(ctx, cells, 48 * sizeof(int64_t)));
    DT_TRY(count_enqueue(g, dq, nullptr, ctx->stream, true, cells.as<int64_t>(), ctx->scratch));
    DT_HIP(hipMemcpyAsync(out, cells.ptr, 48 * sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    DT_HIP(hipStreamSynchronize(ctx->stream));
    return DT_OK;
}

int dt_count_batch(dt_ctx *ctx, uint64_t k, dt_graph *const *graphs, const dt_query *queries,
                   int64_t (*out)[8]) {
    clear_error();
    if (!ctx) return fail(DT_EINVAL, "null context");
    if (k && (!graphs || !queries || !out)) return fail(DT_EINVAL, "null batch array");
    DeviceGuard dg(ctx->device);
    return count_batch(ctx, k, graphs, queries, out);
}

int dt_ctx_batch_tuning(const dt_ctx *ctx, uint32_t out[2]) {
    clear_error();
    if (!ctx || !out) return fail(DT_EINVAL, "null argument");
    out[0] = ctx->batch_tune.light_chunk;
    out[1] = ctx->batch_tune.medium_group;
    return DT_OK;
}

int dt_ctx_set_profiling(dt_ctx *ctx, int enable) {
    clear_error();
    if (!ctx) return fail(DT_EINVAL, "null context");
    DeviceGuard dg(ctx->device);
    if (enable && !ctx->prof_ev[0])
        for (auto &e : ctx->prof_ev) DT_HIP(hipEventCreate(&e));
    ctx->prof = enable != 0;
    for (auto &u : ctx->prof_used) u = false;
    return DT_OK;
}

int dt_ctx_last_profile(dt_ctx *ctx, float ms[DT_PROFILE_SLOTS]) {
    clear_error();
    if (!ctx || !ms) return fail(DT_EINVAL, "null argument");
    DeviceGuard dg(ctx->device);
    for (int i = 0; i < DT_PROFILE_SLOTS; ++i) {
        ms[i] = 0.f;
        if (!ctx->prof_used[i]) continue;
        DT_HIP(hipEventSynchronize(ctx->prof_ev[2 * i + 1]));
        DT_HIP(hipEventElapsedTime(&ms[i], ctx->prof_ev[2 * i], ctx->prof_ev[2 * i + 1]));
    }
    return DT_OK;
}

int dt_graph_order(const dt_graph *g, uint32_t *core, uint32_t *rank) {
    clear_error();
    DT_TRY(check_graph(g, true));
    DeviceGuard dg(g->ctx->device);
    if (core && g->n) DT_HIP(hipMemcpy(core, g->core.ptr, (uint64_t)g->n * 4, hipMemcpyDeviceToHost));
    if (rank && g->n) DT_HIP(hipMemcpy(rank, g->rank.ptr, (uint64_t)g->n * 4, hipMemcpyDeviceToHost));
    return DT_OK;
}

int dt_graph_triangles(const dt_graph *g, uint32_t *out, uint64_t cap, uint64_t *count) {
    clear_error();
    DT_TRY(check_graph(g, true));
    if (!count) return fail(DT_EINVAL, "null count");
    *count = g->n_tri;
    if (!out || cap == 0 || g->n_tri == 0) return DT_OK;
    DeviceGuard dg(g->ctx->device);
    DevMem tri, buf;
    uint64_t ntri = 0, cand = 0, nlist = 0;
    DT_TRY(enumerate_triangles(g, tri, &ntri, &cand, &nlist));
    if (ntri != g->n_tri) return fail(DT_EDEVICE, "triangle enumeration changed between passes");
    DT_TRY(dev_alloc(g->ctx, buf, nlist * 12));
    hipStream_t st = g->ctx->stream;
    k_tri_vertices<<<grid_for(nlist, kBlock), kBlock, 0, st>>>(nlist, tri.as<uint32_t>(), g->n,
        g->dag_row.as<uint32_t>(), g->dag_col.as<uint32_t>(), g->order.as<uint32_t>(), buf.as<uint32_t>());
    DT_HIP(hipGetLastError());
    // the list's triangles without its empty entries
    std::vector<uint32_t> all(3 * nlist);
    DT_HIP(hipMemcpyAsync(all.data(), buf.ptr, nlist * 12, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    uint64_t k = 0;
    for (uint64_t i = 0; i < nlist && k < cap; ++i) {
        if (all[3 * i] == kNoEdge) continue;
        memcpy(out + 3 * k, &all[3 * i], 12);
        ++k;
    }
    return DT_OK;
}

int dt_graph_free(dt_graph *g) {
    clear_error();
    if (!g) return fail(DT_EINVAL, "null graph");
    DeviceGuard dg(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    delete g;
    return DT_OK;
}

}  // extern "C"
