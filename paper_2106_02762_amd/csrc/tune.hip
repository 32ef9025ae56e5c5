// Autotuner of the count: for a graph of a given size class on a given device it picks the light
// rule's pair cap and the weight of the cost model that splits the other triangles between the
// medium path and the prefix procedures (each candidate is a schedule built and timed), then the
// light and medium kernels' blocks per compute unit.  The objective is the geometric mean of the
// whole-span count times at five d13 from ten minutes to infinity (the paper's sweeps of Section 6
// reach eleven days), so that the split serves short and long deltas alike.  Choices are cached per (device, size class) for the process and reused by
// every later build of a graph in that class, by the batched path and by the server (which count
// with the schedules those builds made).  Results never depend on any of these choices.
#include <array>
#include <cmath>
#include <map>

#include "internal.h"

namespace dt {

namespace {

std::mutex g_mu;
std::map<std::array<int, 4>, TunedCount> g_cache;

int ilog2(uint64_t x) {
    int b = 0;
    while (x > 1) {
        x >>= 1;
        ++b;
    }
    return b;
}

// size class: device, and the binary orders of the triangles, temporal edges and the largest
// multiplicity
std::array<int, 4> size_class(const dt_graph *g) {
    return {g->ctx->device, ilog2(g->n_tri), ilog2(g->m), ilog2((uint64_t)g->max_mult + 1)};
}

// the smallest of three event-timed whole-span counts at each d13; the score is the sum of their
// logarithms (the geometric mean's order), so that each delta weighs alike
int time_counts(dt_graph *g, float *ms_out) {
    dt_ctx *ctx = g->ctx;
    const int64_t ds[5] = {600, 3600, 86400, 1000000, INT64_MAX};
    hipEvent_t a = nullptr, b = nullptr;
    DT_HIP(hipEventCreate(&a));
    DT_HIP(hipEventCreate(&b));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{a, b};
    float total = 0.f;
    for (int64_t d : ds) {
        const dt_query qq{d, d, d, INT64_MIN, INT64_MAX};
        DQuery q;
        bool empty = false;
        DT_TRY(normalise_query(g, &qq, &q, &empty));
        if (empty) continue;
        DT_TRY(count_enqueue(g, q, ctx->out8.as<int64_t>(), ctx->stream, false, nullptr, ctx->scratch));
        float best = 1e30f;
        for (int r = 0; r < 3; ++r) {
            DT_HIP(hipEventRecord(a, ctx->stream));
            DT_TRY(count_enqueue(g, q, ctx->out8.as<int64_t>(), ctx->stream, false, nullptr, ctx->scratch));
            DT_HIP(hipEventRecord(b, ctx->stream));
            DT_HIP(hipEventSynchronize(b));
            float ms = 0.f;
            DT_HIP(hipEventElapsedTime(&ms, a, b));
            best = ms < best ? ms : best;
        }
        total += logf(best > 1e-4f ? best : 1e-4f);
    }
    *ms_out = total;
    return DT_OK;
}

}  // namespace

bool tuned_lookup(const dt_graph *g, TunedCount *t) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(size_class(g));
    if (it == g_cache.end()) return false;
    *t = it->second;
    return true;
}

// A candidate replaces the best one so far only when its score is lower by more than kMargin (in
// the sum of the five logarithms: about 2% on the geometric mean), and the defaults are timed first,
// so that candidates within timing noise of each other leave the same choice from run to run.
constexpr float kMargin = 0.1f;

int autotune_count(dt_graph *g, DevMem &tri, TunedCount *out) {
    // the defaults first (light cap 4, weight 100; 16 and 8 blocks per CU)
    const uint32_t caps[3] = {4, 2, 8}, pcts[3] = {100, 25, 400};
    TunedCount best;
    float best_ms = 1e30f;
    g->geom = CountGeom();
    for (uint32_t lc : caps)
        for (uint32_t cp : pcts) {
            g->light_cap_used = lc;
            g->cost_pct_used = cp;
            DT_TRY(make_schedule(g, tri));
            float ms = 0.f;
            DT_TRY(time_counts(g, &ms));
            if (ms < best_ms - kMargin) {
                best_ms = ms;
                best.light_cap = lc;
                best.cost_pct = cp;
            }
        }
    g->light_cap_used = best.light_cap;
    g->cost_pct_used = best.cost_pct;
    DT_TRY(make_schedule(g, tri));
    const uint32_t lbpc[3] = {16, 8, 32}, mbpc[3] = {8, 4, 16};
    best_ms = 1e30f;
    for (uint32_t l : lbpc)
        for (uint32_t m : mbpc) {
            g->geom.light_bpc = l;
            g->geom.medium_bpc = m;
            float ms = 0.f;
            DT_TRY(time_counts(g, &ms));
            if (ms < best_ms - kMargin) {
                best_ms = ms;
                best.light_bpc = l;
                best.medium_bpc = m;
            }
        }
    g->geom.light_bpc = best.light_bpc;
    g->geom.medium_bpc = best.medium_bpc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[size_class(g)] = best;
    }
    *out = best;
    return DT_OK;
}

}  // namespace dt
