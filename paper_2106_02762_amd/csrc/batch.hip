// Batched counting: many (graph, query) pairs in one call.
#include "internal.h"

namespace dt {

int count_batch(dt_ctx *ctx, uint64_t k, dt_graph *const *graphs, const dt_query *queries,
                int64_t (*out)[8]) {
    if (k == 0) return DT_OK;
    DevMem outs;
    DT_TRY(dev_alloc(ctx, outs, k * 8 * sizeof(int64_t)));
    hipStream_t s = ctx->stream;
    DT_HIP(hipMemsetAsync(outs.ptr, 0, k * 8 * sizeof(int64_t), s));
    for (uint64_t i = 0; i < k; ++i) {
        dt_graph *g = graphs[i];
        if (!g || g->ctx != ctx) return fail(DT_EINVAL, "batch entry %llu: graph of another context", (unsigned long long)i);
        if (!g->built) return fail(DT_ENOTBUILT, "batch entry %llu: graph not built", (unsigned long long)i);
        DQuery dq;
        bool empty = false;
        DT_TRY(normalise_query(g, &queries[i], &dq, &empty));
        if ((g->sum_sigma3 >> 63) != 0) return fail(DT_EOVERFLOW, "batch entry %llu may overflow", (unsigned long long)i);
        if (empty || g->n_tri == 0) continue;
        DT_TRY(count_enqueue(g, dq, outs.as<int64_t>() + 8 * i, s, false, nullptr));
    }
    DT_HIP(hipMemcpyAsync(out, outs.ptr, k * 8 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DT_HIP(hipStreamSynchronize(s));
    return DT_OK;
}

}  // namespace dt
