// Orientation of G by the degeneracy ordering into the DAG G_prec (Section 3: orient {u, v} from
// u to v iff u comes first), and the re-layout of the temporal edge store in DAG-edge order.
//
// Vertices are renamed by their rank, so a DAG edge is (rank u, rank v) with rank u < rank v and
// the out-neighbours of u are a sorted run.  DAG edges are numbered in (tail, head) order, and the
// temporal edges of DAG edge d are stored at [eoff[2d], eoff[2d+2]): first those directed
// tail -> head, then head -> tail, each in key order (a scatter by rank, no re-sort).  All edges at one source vertex u are then
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

// DAG edge d (in (tail, head) order) is pair s = dv[d]: its head rank, the pair's DAG id and
// direction swap, the sizes of its two direction groups, and the CSR rows: the edges being sorted
// by tail, dag_row[u] for every u in (tail of d - 1, tail of d] is d (d = ms closes the array)
__global__ void k_dag_fill(uint64_t ms, uint32_t n, const uint64_t *__restrict__ dk,
                           const uint32_t *__restrict__ dv, const uint32_t *__restrict__ sx,
                           const uint32_t *__restrict__ rank, const uint32_t *__restrict__ pstart,
                           const uint32_t *__restrict__ c1, uint32_t *__restrict__ dag_col,
                           uint32_t *__restrict__ dag_of, uint8_t *__restrict__ sflip,
                           uint32_t *__restrict__ dag_row, uint32_t *__restrict__ gsize) {
    uint64_t d = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (d > ms) return;
    const uint32_t tail = d < ms ? (uint32_t)(dk[d] >> 32) : n;
    const int64_t prev = d > 0 ? (int64_t)(dk[d - 1] >> 32) : -1;
    for (int64_t u = prev + 1; u <= (int64_t)tail; ++u) dag_row[u] = (uint32_t)d;
    if (d == ms) return;
    const uint64_t k = dk[d];
    const uint32_t s = dv[d];
    dag_col[d] = (uint32_t)k;
    dag_of[s] = (uint32_t)d;
    // pdir = 0 means sx -> sy; the DAG tail is sx unless sx has the larger rank
    const uint32_t flip = rank[sx[s]] != tail ? 1u : 0u;
    sflip[s] = (uint8_t)flip;
    const uint32_t ps = pstart[s], pe = pstart[s + 1];
    const uint32_t n1 = c1[pe] - c1[ps], n0 = (pe - ps) - n1;
    gsize[2 * d] = flip ? n1 : n0;       // tail -> head
    gsize[2 * d + 1] = flip ? n0 : n1;   // head -> tail
}

// largest out-degree: max of row[i + 1] - row[i] over i < n
__global__ void k_max_u32(uint64_t n, const uint32_t *__restrict__ row, unsigned *__restrict__ out) {
    __shared__ unsigned s[kBlock];
    unsigned mx = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) {
        const unsigned dg = row[i + 1] - row[i];
        mx = dg > mx ? dg : mx;
    }
    s[threadIdx.x] = mx;
    __syncthreads();
    for (unsigned w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, s[0]);
}

// Move every temporal edge (pair-major, key order within the pair) to its place in the DAG-edge
// layout: group 2d + direction, at its rank among the pair's edges of that direction.  Ranks come
// from the running count c1 of head->tail flags, so each group stays in key order.
__global__ void k_relayout(uint64_t m, const uint32_t *__restrict__ psid, const uint8_t *__restrict__ pdir,
                           const uint32_t *__restrict__ pstart, const uint32_t *__restrict__ c1,
                           const uint32_t *__restrict__ dag_of, const uint8_t *__restrict__ sflip,
                           const uint32_t *__restrict__ eoff, const uint64_t *__restrict__ pkey,
                           uint64_t *__restrict__ key) {
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m) return;
    const uint32_t s = psid[k], ps = pstart[s], dir = pdir[k];
    const uint32_t ones = c1[k] - c1[ps];
    const uint32_t r = dir ? ones : (uint32_t)(k - ps) - ones;
    const uint32_t g = 2 * dag_of[s] + (dir ^ sflip[s]);
    key[eoff[g] + r] = pkey[k];
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
    DevMem dk, dv, dk2, dv2, dag_of, sflip, gsize, scal;
    const uint64_t ngroups = 2 * ms;
    DT_TRY(dev_alloc(ctx, dk, ms * 8));
    DT_TRY(dev_alloc(ctx, dv, ms * 4));
    DT_TRY(dev_alloc(ctx, dk2, ms * 8));
    DT_TRY(dev_alloc(ctx, dv2, ms * 4));
    DT_TRY(dev_alloc(ctx, dag_of, ms * 4));
    DT_TRY(dev_alloc(ctx, sflip, ms));
    DT_TRY(dev_alloc(ctx, gsize, (ngroups + 1) * 4));
    DT_TRY(dev_alloc(ctx, g->dag_col, ms * 4));
    DT_TRY(dev_alloc(ctx, g->dag_row, ((uint64_t)n + 1) * 4));
    DT_TRY(dev_alloc(ctx, g->eoff, (ngroups + 1) * 4));
    DT_TRY(dev_alloc(ctx, g->key, m * 8));
    DT_TRY(dev_alloc(ctx, scal, 256));
    DT_HIP(hipMemsetAsync(gsize.ptr, 0, (ngroups + 1) * 4, st));
    DT_HIP(hipMemsetAsync(scal.ptr, 0, 256, st));
    if (ms) {
        k_dag_keys<<<grid_for(ms, kBlock), kBlock, 0, st>>>(ms, g->sx.as<uint32_t>(), g->sy.as<uint32_t>(),
                                                            g->rank.as<uint32_t>(), dk.as<uint64_t>(),
                                                            dv.as<uint32_t>());
        DT_HIP(hipGetLastError());
        DT_TRY(sort_pairs_u64_u32(ctx, dk.as<uint64_t>(), dk2.as<uint64_t>(), dv.as<uint32_t>(),
                                  dv2.as<uint32_t>(), ms, 32 + bits_for((uint64_t)n + 1), st));
    }
    k_dag_fill<<<grid_for(ms + 1, kBlock), kBlock, 0, st>>>(
        ms, n, dk2.as<uint64_t>(), dv2.as<uint32_t>(), g->sx.as<uint32_t>(), g->rank.as<uint32_t>(),
        g->pstart.as<uint32_t>(), g->c1.as<uint32_t>(), g->dag_col.as<uint32_t>(), dag_of.as<uint32_t>(),
        sflip.as<uint8_t>(), g->dag_row.as<uint32_t>(), gsize.as<uint32_t>());
    DT_HIP(hipGetLastError());
    if (n) {
        unsigned grid = grid_for(n, kBlock);
        if (grid > 2048) grid = 2048;
        k_max_u32<<<grid, kBlock, 0, st>>>(n, g->dag_row.as<uint32_t>(), scal.as<unsigned>());
        DT_HIP(hipGetLastError());
    }
    DT_TRY(exclusive_scan_u32(ctx, gsize.as<uint32_t>(), g->eoff.as<uint32_t>(), ngroups + 1, st));
    if (m) {
        prof_begin(ctx, kProfRelayout, st);
        k_relayout<<<grid_for(m, kBlock), kBlock, 0, st>>>(m, g->psid.as<uint32_t>(), g->pdir.as<uint8_t>(),
            g->pstart.as<uint32_t>(), g->c1.as<uint32_t>(), dag_of.as<uint32_t>(), sflip.as<uint8_t>(),
            g->eoff.as<uint32_t>(), g->pkey.as<uint64_t>(), g->key.as<uint64_t>());
        prof_end(ctx, kProfRelayout, st);
        DT_HIP(hipGetLastError());
    }
    unsigned mo = 0;
    DT_HIP(hipMemcpyAsync(&mo, scal.ptr, 4, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    g->max_outdeg = mo;
    return DT_OK;
}

}  // namespace dt
