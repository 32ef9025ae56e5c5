// Count schedule, built once per graph (it does not depend on the deltas, Section 6 "running time
// independent of time periods"): each static triangle goes to the light path (one lane) or the
// heavy path (the prefix-count procedures split over workgroups), decided by how many
// (uv edge, uw edge) pairs the light path would walk.  Also the graph totals reported in the
// statistics: the sum over triangles of the product of the three pair multiplicities (the count at
// infinite deltas, an overflow bound) and the algorithmic bytes of one whole-graph count.
#include "internal.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;

__device__ __forceinline__ uint32_t ceil_log2_1(uint32_t s) {   // ceil(log2(s + 1))
    return s == 0 ? 0 : 32 - __clz(s);
}

// per triangle: heavy flag; per block: sum of sigma products (128-bit as two words) and bytes
__global__ void k_classify(uint64_t n_tri, const uint32_t *__restrict__ tri, const uint32_t *__restrict__ eoff,
                           uint64_t cap, uint64_t *__restrict__ hflag, uint64_t *__restrict__ part) {
    __shared__ unsigned long long s_lo[kBlock], s_hi[kBlock], s_b[kBlock];
    unsigned __int128 acc = 0;
    unsigned long long bytes = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n_tri; i += (uint64_t)gridDim.x * kBlock) {
        const uint32_t e_uv = tri[3 * i], e_uw = tri[3 * i + 1], e_vw = tri[3 * i + 2];
        const uint64_t s_uv = eoff[2 * e_uv + 2] - eoff[2 * e_uv];
        const uint64_t s_uw = eoff[2 * e_uw + 2] - eoff[2 * e_uw];
        const uint32_t s_vw = eoff[2 * e_vw + 2] - eoff[2 * e_vw];
        hflag[i] = (s_uv * s_uw > cap) ? 1ull : 0ull;
        acc += (unsigned __int128)(s_uv * s_uw) * s_vw;
        const uint32_t probe = 2 * ceil_log2_1(s_vw);
        bytes += 12 + 36 + 8 * (s_uv + s_uw) + 8 * (uint64_t)(s_vw < probe ? s_vw : probe);
    }
    s_lo[threadIdx.x] = (unsigned long long)acc;
    s_hi[threadIdx.x] = (unsigned long long)(acc >> 64);
    s_b[threadIdx.x] = bytes;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned __int128 t = 0;
        unsigned long long b = 0;
        for (unsigned j = 0; j < kBlock; ++j) {
            t += ((unsigned __int128)s_hi[j] << 64) | s_lo[j];
            b += s_b[j];
        }
        part[3 * blockIdx.x] = (uint64_t)t;
        part[3 * blockIdx.x + 1] = (uint64_t)(t >> 64);
        part[3 * blockIdx.x + 2] = b;
    }
}

__global__ void k_partition(uint64_t n_tri, const uint32_t *__restrict__ tri, const uint64_t *__restrict__ hflag,
                            const uint64_t *__restrict__ hpos, uint32_t *__restrict__ light,
                            uint32_t *__restrict__ heavy) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_tri) return;
    uint32_t *dst = hflag[i] ? heavy + 3 * hpos[i] : light + 3 * (i - hpos[i]);
    dst[0] = tri[3 * i];
    dst[1] = tri[3 * i + 1];
    dst[2] = tri[3 * i + 2];
}

// slots (four prefix arrays of length sigma + 1) and chunks of every heavy triangle
__global__ void k_heavy_sizes(uint64_t n_heavy, const uint32_t *__restrict__ heavy,
                              const uint32_t *__restrict__ eoff, uint32_t chunk,
                              uint64_t *__restrict__ slots, uint64_t *__restrict__ nch) {
    uint64_t h = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (h >= n_heavy) return;
    const uint32_t e_uv = heavy[3 * h], e_uw = heavy[3 * h + 1];
    const uint64_t src = (uint64_t)(eoff[2 * e_uv + 2] - eoff[2 * e_uv]) + (eoff[2 * e_uw + 2] - eoff[2 * e_uw]);
    slots[h] = src + 4;
    nch[h] = (src + chunk - 1) / chunk;
}

__global__ void k_heavy_chunks(uint64_t n_heavy, const uint64_t *__restrict__ nch,
                               const uint64_t *__restrict__ cbase, uint32_t chunk,
                               uint32_t *__restrict__ chunks) {
    uint64_t h = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (h >= n_heavy) return;
    for (uint64_t j = 0; j < nch[h]; ++j) {
        chunks[2 * (cbase[h] + j)] = (uint32_t)h;
        chunks[2 * (cbase[h] + j) + 1] = (uint32_t)(j * chunk);
    }
}

}  // namespace

int make_schedule(dt_graph *g, DevMem &tri) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint64_t nt = g->n_tri;
    Schedule &S = g->sched;
    S = Schedule();
    const uint64_t cap = g->tuning.force_path == 1 ? ~0ull
                       : g->tuning.force_path == 2 ? 0ull : (uint64_t)g->tuning.light_pair_cap;
    const uint32_t chunk = g->tuning.heavy_chunk;
    DevMem hflag, hpos, part;
    DT_TRY(dev_alloc(ctx, hflag, (nt + 1) * 8));
    DT_TRY(dev_alloc(ctx, hpos, (nt + 1) * 8));
    unsigned grid = grid_for(nt, kBlock);
    if (grid > 4096) grid = 4096;
    DT_TRY(dev_alloc(ctx, part, (uint64_t)grid * 3 * 8));
    DT_HIP(hipMemsetAsync(hflag.ptr, 0, (nt + 1) * 8, st));
    k_classify<<<grid, kBlock, 0, st>>>(nt, tri.as<uint32_t>(), g->eoff.as<uint32_t>(), cap,
                                        hflag.as<uint64_t>(), part.as<uint64_t>());
    DT_HIP(hipGetLastError());
    std::vector<uint64_t> hp((size_t)grid * 3);
    DT_HIP(hipMemcpyAsync(hp.data(), part.ptr, hp.size() * 8, hipMemcpyDeviceToHost, st));
    DT_TRY(exclusive_scan_u64(ctx, hflag.as<uint64_t>(), hpos.as<uint64_t>(), nt + 1, st));
    uint64_t nh = 0;
    DT_HIP(hipMemcpyAsync(&nh, hpos.as<uint64_t>() + nt, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    unsigned __int128 s3 = 0;
    uint64_t bytes = 0;
    for (unsigned b = 0; b < grid; ++b) {
        s3 += ((unsigned __int128)hp[3 * b + 1] << 64) | hp[3 * b];
        bytes += hp[3 * b + 2];
    }
    g->sum_sigma3 = s3;
    g->alg_bytes = bytes;
    S.n_heavy = nh;
    S.n_light = nt - nh;
    DT_TRY(dev_alloc(ctx, S.light, S.n_light * 12));
    DT_TRY(dev_alloc(ctx, S.heavy, S.n_heavy * 12));
    if (nt) {
        k_partition<<<grid_for(nt, kBlock), kBlock, 0, st>>>(nt, tri.as<uint32_t>(), hflag.as<uint64_t>(),
                                                             hpos.as<uint64_t>(), S.light.as<uint32_t>(),
                                                             S.heavy.as<uint32_t>());
        DT_HIP(hipGetLastError());
    }
    DT_HIP(hipStreamSynchronize(st));
    hflag.reset();
    hpos.reset();
    // heavy slots and chunks
    DevMem slots, nch, cbase;
    DT_TRY(dev_alloc(ctx, slots, (nh + 1) * 8));
    DT_TRY(dev_alloc(ctx, nch, (nh + 1) * 8));
    DT_TRY(dev_alloc(ctx, cbase, (nh + 1) * 8));
    DT_TRY(dev_alloc(ctx, S.hslot, (nh + 1) * 8));
    DT_HIP(hipMemsetAsync(slots.ptr, 0, (nh + 1) * 8, st));
    DT_HIP(hipMemsetAsync(nch.ptr, 0, (nh + 1) * 8, st));
    if (nh) {
        k_heavy_sizes<<<grid_for(nh, kBlock), kBlock, 0, st>>>(nh, S.heavy.as<uint32_t>(), g->eoff.as<uint32_t>(),
                                                               chunk, slots.as<uint64_t>(), nch.as<uint64_t>());
        DT_HIP(hipGetLastError());
    }
    DT_TRY(exclusive_scan_u64(ctx, slots.as<uint64_t>(), S.hslot.as<uint64_t>(), nh + 1, st));
    DT_TRY(exclusive_scan_u64(ctx, nch.as<uint64_t>(), cbase.as<uint64_t>(), nh + 1, st));
    uint64_t tot[2] = {0, 0};
    DT_HIP(hipMemcpyAsync(&tot[0], S.hslot.as<uint64_t>() + nh, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipMemcpyAsync(&tot[1], cbase.as<uint64_t>() + nh, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    S.n_slots = tot[0];
    S.n_chunks = tot[1];
    if (S.n_chunks > 0xffffffffull || nh > 0xffffffffull)
        return fail(DT_EOVERFLOW, "too many heavy work items (%llu)", (unsigned long long)S.n_chunks);
    DT_TRY(dev_alloc(ctx, S.chunks, S.n_chunks * 8));
    if (nh) {
        k_heavy_chunks<<<grid_for(nh, kBlock), kBlock, 0, st>>>(nh, nch.as<uint64_t>(), cbase.as<uint64_t>(),
                                                                chunk, S.chunks.as<uint32_t>());
        DT_HIP(hipGetLastError());
    }
    DT_HIP(hipStreamSynchronize(st));
    return DT_OK;
}

}  // namespace dt
