// Orientation of G by the degeneracy ordering into the DAG G_prec (Section 3: orient {u, v} from
// u to v iff u comes first), and the re-layout of the temporal edge store in DAG-edge order.
//
// Vertices are renamed by their rank, so a DAG edge is (rank u, rank v) with rank u < rank v and
// the out-neighbours of u are a sorted run.  DAG edges are numbered in (tail, head) order, and the
// temporal edges of DAG edge d are stored at [eoff[2d], eoff[2d+2]): first those directed
// tail -> head, then head -> tail, each in key order.  All edges at one source vertex u are then
// one contiguous stretch of the store, which is exactly what the counting of all triangles with
// source u walks (Section 5: only {u,v} and {u,w} are enumerated).
#include "internal.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;

__global__ void k_dag_keys(uint64_t ms, const uint32_t *__restrict__ sx, const uint32_t *__restrict__ sy,
                           const uint32_t *__restrict__ rank, uint64_t *__restrict__ dk,
                           uint32_t *__restrict__ dv) {
    uint64_t s = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= ms) return;
    uint32_t rx = rank[sx[s]], ry = rank[sy[s]];
    uint32_t a = rx < ry ? rx : ry, b = rx < ry ? ry : rx;
    dk[s] = ((uint64_t)a << 32) | b;
    dv[s] = (uint32_t)s;
}

__global__ void k_dag_fill(uint64_t ms, const uint64_t *__restrict__ dk, const uint32_t *__restrict__ dv,
                           uint32_t *__restrict__ dag_col, uint32_t *__restrict__ dag_of,
                           uint32_t *__restrict__ outdeg) {
    uint64_t d = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (d >= ms) return;
    uint64_t k = dk[d];
    dag_col[d] = (uint32_t)k;
    dag_of[dv[d]] = (uint32_t)d;
    atomicAdd(&outdeg[(uint32_t)(k >> 32)], 1u);
}

__global__ void k_max_u32(uint64_t n, const uint32_t *__restrict__ a, unsigned *__restrict__ out) {
    __shared__ unsigned s[kBlock];
    unsigned mx = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock)
        mx = a[i] > mx ? a[i] : mx;
    s[threadIdx.x] = mx;
    __syncthreads();
    for (unsigned w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, s[0]);
}

// group of each temporal edge in the new layout: 2 * dag_edge + (0 tail->head, 1 head->tail)
__global__ void k_group_keys(uint64_t m, const uint32_t *__restrict__ psid, const uint8_t *__restrict__ pdir,
                             const uint32_t *__restrict__ sx, const uint32_t *__restrict__ sy,
                             const uint32_t *__restrict__ rank, const uint32_t *__restrict__ dag_of,
                             uint64_t *__restrict__ gk, uint32_t *__restrict__ gcount) {
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m) return;
    uint32_t s = psid[k];
    // pdir = 0: edge goes sx -> sy.  The DAG tail is sx iff rank[sx] < rank[sy].
    uint32_t flip = rank[sx[s]] > rank[sy[s]] ? 1u : 0u;
    uint32_t dir = (uint32_t)pdir[k] ^ flip;
    uint64_t g = 2 * (uint64_t)dag_of[s] + dir;
    gk[k] = g;
    atomicAdd(&gcount[g], 1u);
}

int bits_for(uint64_t x) {
    int b = 1;
    while (b < 64 && (1ull << b) < x) b++;
    return b;
}

}  // namespace

int orient(dt_graph *g) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint64_t ms = g->m_s, m = g->m;
    const uint32_t n = g->n;
    DevMem dk, dv, dk2, dv2, dag_of, outdeg, scal;
    DT_TRY(dev_alloc(ctx, dk, ms * 8));
    DT_TRY(dev_alloc(ctx, dv, ms * 4));
    DT_TRY(dev_alloc(ctx, dk2, ms * 8));
    DT_TRY(dev_alloc(ctx, dv2, ms * 4));
    DT_TRY(dev_alloc(ctx, dag_of, ms * 4));
    DT_TRY(dev_alloc(ctx, outdeg, ((uint64_t)n + 1) * 4));
    DT_TRY(dev_alloc(ctx, g->dag_col, ms * 4));
    DT_TRY(dev_alloc(ctx, g->dag_row, ((uint64_t)n + 1) * 4));
    DT_TRY(dev_alloc(ctx, scal, 256));
    DT_HIP(hipMemsetAsync(outdeg.ptr, 0, ((uint64_t)n + 1) * 4, st));
    DT_HIP(hipMemsetAsync(scal.ptr, 0, 256, st));
    if (ms) {
        k_dag_keys<<<grid_for(ms, kBlock), kBlock, 0, st>>>(ms, g->sx.as<uint32_t>(), g->sy.as<uint32_t>(),
                                                            g->rank.as<uint32_t>(), dk.as<uint64_t>(),
                                                            dv.as<uint32_t>());
        DT_HIP(hipGetLastError());
        DT_TRY(sort_pairs_u64_u32(ctx, dk.as<uint64_t>(), dk2.as<uint64_t>(), dv.as<uint32_t>(),
                                  dv2.as<uint32_t>(), ms, 32 + bits_for((uint64_t)n + 1), st));
        k_dag_fill<<<grid_for(ms, kBlock), kBlock, 0, st>>>(ms, dk2.as<uint64_t>(), dv2.as<uint32_t>(),
                                                            g->dag_col.as<uint32_t>(), dag_of.as<uint32_t>(),
                                                            outdeg.as<uint32_t>());
        DT_HIP(hipGetLastError());
        unsigned grid = grid_for(n, kBlock);
        if (grid > 2048) grid = 2048;
        k_max_u32<<<grid, kBlock, 0, st>>>(n, outdeg.as<uint32_t>(), scal.as<unsigned>());
        DT_HIP(hipGetLastError());
    }
    DT_TRY(exclusive_scan_u32(ctx, outdeg.as<uint32_t>(), g->dag_row.as<uint32_t>(), (uint64_t)n + 1, st));
    unsigned mo = 0;
    DT_HIP(hipMemcpyAsync(&mo, scal.ptr, 4, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    g->max_outdeg = mo;
    dk.reset(); dv.reset(); dk2.reset(); dv2.reset(); outdeg.reset();

    // temporal store in DAG-edge order; the sort is stable, so each group keeps key order
    DevMem gk, gk2, gcount;
    const uint64_t ngroups = 2 * ms;
    DT_TRY(dev_alloc(ctx, gk, m * 8));
    DT_TRY(dev_alloc(ctx, gk2, m * 8));
    DT_TRY(dev_alloc(ctx, gcount, (ngroups + 1) * 4));
    DT_TRY(dev_alloc(ctx, g->key, m * 8));
    DT_TRY(dev_alloc(ctx, g->eoff, (ngroups + 1) * 4));
    DT_HIP(hipMemsetAsync(gcount.ptr, 0, (ngroups + 1) * 4, st));
    if (m) {
        k_group_keys<<<grid_for(m, kBlock), kBlock, 0, st>>>(m, g->psid.as<uint32_t>(), g->pdir.as<uint8_t>(),
                                                             g->sx.as<uint32_t>(), g->sy.as<uint32_t>(),
                                                             g->rank.as<uint32_t>(), dag_of.as<uint32_t>(),
                                                             gk.as<uint64_t>(), gcount.as<uint32_t>());
        DT_HIP(hipGetLastError());
        DT_TRY(sort_pairs_u64_u64(ctx, gk.as<uint64_t>(), gk2.as<uint64_t>(), g->pkey.as<uint64_t>(),
                                  g->key.as<uint64_t>(), m, bits_for(ngroups + 1), st));
    }
    DT_TRY(exclusive_scan_u32(ctx, gcount.as<uint32_t>(), g->eoff.as<uint32_t>(), ngroups + 1, st));
    DT_HIP(hipStreamSynchronize(st));
    return DT_OK;
}

}  // namespace dt
