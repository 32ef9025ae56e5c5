// Static triangle enumeration in G_prec (Section 5 and the proof of Theorem 1): for every DAG
// edge (u, v) and every w in N+(u), {u, v, w} is a triangle iff w is also in N+(v); u is then the
// source vertex and u < v < w in the ordering.  The paper tests {v, w} with a hash lookup; here
// N+(u) after v and N+(v) are both sorted runs of at most degeneracy entries, and the shorter is
// binary-searched in the longer, which yields the DAG edge ids of {u, w} and {v, w} directly.
//
// Two passes (count, exclusive scan, fill) so that the list is written in (u, v) order with no
// atomics: triangles sharing a source vertex are adjacent, as are their edge lists in the store.
#include "internal.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;

__global__ void k_tails(uint32_t n, const uint32_t *__restrict__ dag_row, uint32_t *__restrict__ tail) {
    uint32_t u = blockIdx.x * kBlock + threadIdx.x;
    if (u >= n) return;
    for (uint32_t d = dag_row[u]; d < dag_row[u + 1]; ++d) tail[d] = u;
}

__device__ __forceinline__ uint32_t find_u32(const uint32_t *__restrict__ a, uint32_t lo, uint32_t hi,
                                             uint32_t x) {
    uint32_t len = hi - lo;
    while (len > 0) {
        uint32_t half = len >> 1;
        if (a[lo + half] < x) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

// For DAG edge d = (u, v): common entries of N+(u) after v (positions d+1 .. row[u+1]) and N+(v).
template <bool FILL>
__global__ void k_tri(uint64_t ms, const uint32_t *__restrict__ dag_row, const uint32_t *__restrict__ dag_col,
                      const uint32_t *__restrict__ tail, uint64_t *__restrict__ cnt,
                      const uint64_t *__restrict__ off, uint32_t *__restrict__ tri) {
    uint64_t d = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (d >= ms) return;
    const uint32_t u = tail[d], v = dag_col[d];
    const uint32_t a0 = (uint32_t)d + 1, a1 = dag_row[u + 1];
    const uint32_t b0 = dag_row[v], b1 = dag_row[v + 1];
    uint64_t c = 0;
    uint64_t o = FILL ? off[d] : 0;
    if (a1 > a0 && b1 > b0) {
        const bool a_short = (a1 - a0) <= (b1 - b0);
        const uint32_t s0 = a_short ? a0 : b0, s1 = a_short ? a1 : b1;
        uint32_t l0 = a_short ? b0 : a0;
        const uint32_t l1 = a_short ? b1 : a1;
        for (uint32_t i = s0; i < s1 && l0 < l1; ++i) {
            const uint32_t w = dag_col[i];
            const uint32_t j = find_u32(dag_col, l0, l1, w);   // runs are sorted: restart at j
            l0 = j;
            if (j < l1 && dag_col[j] == w) {
                if (FILL) {
                    const uint32_t e_uw = a_short ? i : j, e_vw = a_short ? j : i;
                    tri[3 * (o + c)] = (uint32_t)d;
                    tri[3 * (o + c) + 1] = e_uw;
                    tri[3 * (o + c) + 2] = e_vw;
                }
                ++c;
            }
        }
    }
    if (!FILL) cnt[d] = c;
}

}  // namespace

int enumerate_triangles(dt_graph *g, DevMem &tri) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint64_t ms = g->m_s;
    const uint32_t n = g->n;
    DevMem tail, cnt, off;
    DT_TRY(dev_alloc(ctx, tail, ms * 4));
    DT_TRY(dev_alloc(ctx, cnt, (ms + 1) * 8));
    DT_TRY(dev_alloc(ctx, off, (ms + 1) * 8));
    DT_HIP(hipMemsetAsync(cnt.ptr, 0, (ms + 1) * 8, st));
    if (n) {
        k_tails<<<grid_for(n, kBlock), kBlock, 0, st>>>(n, g->dag_row.as<uint32_t>(), tail.as<uint32_t>());
        DT_HIP(hipGetLastError());
    }
    if (ms) {
        k_tri<false><<<grid_for(ms, kBlock), kBlock, 0, st>>>(ms, g->dag_row.as<uint32_t>(),
            g->dag_col.as<uint32_t>(), tail.as<uint32_t>(), cnt.as<uint64_t>(), nullptr, nullptr);
        DT_HIP(hipGetLastError());
    }
    DT_TRY(exclusive_scan_u64(ctx, cnt.as<uint64_t>(), off.as<uint64_t>(), ms + 1, st));
    uint64_t ntri = 0;
    DT_HIP(hipMemcpyAsync(&ntri, off.as<uint64_t>() + ms, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    g->n_tri = ntri;
    DT_TRY(dev_alloc(ctx, tri, ntri * 12));
    if (ms && ntri) {
        k_tri<true><<<grid_for(ms, kBlock), kBlock, 0, st>>>(ms, g->dag_row.as<uint32_t>(),
            g->dag_col.as<uint32_t>(), tail.as<uint32_t>(), nullptr, off.as<uint64_t>(), tri.as<uint32_t>());
        DT_HIP(hipGetLastError());
    }
    DT_HIP(hipStreamSynchronize(st));
    return DT_OK;
}

}  // namespace dt
