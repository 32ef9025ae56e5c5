// Count schedule, built once per graph (it does not depend on the deltas, Section 6 "running time
// independent of time periods"): each static triangle goes to the light path (one lane), the
// medium path (one wavefront) or the heavy path (the prefix-count procedures split over
// workgroups), decided by P = sigma_uv * sigma_uw, the number of (uv edge, uw edge) pairs the
// pairwise paths walk.  A medium triangle becomes ceil(P / kMediumChunk) work items of equal size.  Also the graph totals reported in the
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
// class 0 light, 1 medium, 2 heavy; force: 0 by the caps, 1 light, 2 heavy, 3 medium
__device__ __forceinline__ int tri_class(uint64_t P, uint64_t cap_l, uint64_t cap_m, uint32_t force) {
    if (force == 1) return 0;
    if (force == 2) return 2;
    if (force == 3) return P < (1ull << 31) ? 1 : 2;
    return P <= cap_l ? 0 : (P <= cap_m ? 1 : 2);
}

__global__ void k_classify(uint64_t n_tri, const uint32_t *__restrict__ tri, const uint32_t *__restrict__ eoff,
                           uint64_t cap_l, uint64_t cap_m, uint32_t force, uint64_t *__restrict__ f1,
                           uint64_t *__restrict__ f2, uint64_t *__restrict__ part) {
    __shared__ unsigned long long s_lo[kBlock], s_hi[kBlock], s_b[kBlock], s_bl[kBlock], s_bm[kBlock];
    unsigned __int128 acc = 0;
    unsigned long long bytes = 0, bytes_light = 0, bytes_medium = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n_tri; i += (uint64_t)gridDim.x * kBlock) {
        const uint32_t e_uv = tri[3 * i], e_uw = tri[3 * i + 1], e_vw = tri[3 * i + 2];
        const uint64_t s_uv = eoff[2 * e_uv + 2] - eoff[2 * e_uv];
        const uint64_t s_uw = eoff[2 * e_uw + 2] - eoff[2 * e_uw];
        const uint32_t s_vw = eoff[2 * e_vw + 2] - eoff[2 * e_vw];
        const int cls = tri_class(s_uv * s_uw, cap_l, cap_m, force);
        const bool heavy = cls != 0;   // bytes_light counts the light class only
        f1[i] = cls == 1 ? 1ull : 0ull;
        f2[i] = cls == 2 ? 1ull : 0ull;
        acc += (unsigned __int128)(s_uv * s_uw) * s_vw;
        const uint32_t probe = 2 * ceil_log2_1(s_vw);
        const uint64_t b = 12 + 36 + 8 * (s_uv + s_uw) + 8 * (uint64_t)(s_vw < probe ? s_vw : probe);
        bytes += b;
        bytes_light += heavy ? 0 : b;
        bytes_medium += cls == 1 ? b : 0;
    }
    s_lo[threadIdx.x] = (unsigned long long)acc;
    s_hi[threadIdx.x] = (unsigned long long)(acc >> 64);
    s_b[threadIdx.x] = bytes;
    s_bl[threadIdx.x] = bytes_light;
    s_bm[threadIdx.x] = bytes_medium;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned __int128 t = 0;
        unsigned long long b = 0, bl = 0, bm = 0;
        for (unsigned j = 0; j < kBlock; ++j) {
            t += ((unsigned __int128)s_hi[j] << 64) | s_lo[j];
            b += s_b[j];
            bl += s_bl[j];
            bm += s_bm[j];
        }
        part[5 * blockIdx.x] = (uint64_t)t;
        part[5 * blockIdx.x + 1] = (uint64_t)(t >> 64);
        part[5 * blockIdx.x + 2] = b;
        part[5 * blockIdx.x + 3] = bl;
        part[5 * blockIdx.x + 4] = bm;
    }
}

__global__ void k_partition(uint64_t n_tri, const uint32_t *__restrict__ tri, const uint64_t *__restrict__ f1,
                            const uint64_t *__restrict__ f2, const uint64_t *__restrict__ p1,
                            const uint64_t *__restrict__ p2, uint32_t *__restrict__ light,
                            uint32_t *__restrict__ medium, uint32_t *__restrict__ heavy) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_tri) return;
    uint32_t *dst = f2[i] ? heavy + 3 * p2[i] : (f1[i] ? medium + 3 * p1[i] : light + 3 * (i - p1[i] - p2[i]));
    dst[0] = tri[3 * i];
    dst[1] = tri[3 * i + 1];
    dst[2] = tri[3 * i + 2];
}

// work items of the medium path: ceil(P / kMediumChunk) per triangle
__global__ void k_medium_sizes(uint64_t nm, const uint32_t *__restrict__ med, const uint32_t *__restrict__ eoff,
                               uint64_t *__restrict__ nch) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nm) return;
    const uint32_t e_uv = med[3 * i], e_uw = med[3 * i + 1];
    const uint64_t P = (uint64_t)(eoff[2 * e_uv + 2] - eoff[2 * e_uv]) * (eoff[2 * e_uw + 2] - eoff[2 * e_uw]);
    nch[i] = (P + kMediumChunk - 1) / kMediumChunk;
}

__global__ void k_medium_fill(uint64_t nm, const uint64_t *__restrict__ nch, const uint64_t *__restrict__ base,
                              uint32_t *__restrict__ items) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nm) return;
    for (uint64_t j = 0; j < nch[i]; ++j) {
        items[2 * (base[i] + j)] = (uint32_t)i;
        items[2 * (base[i] + j) + 1] = (uint32_t)(j * kMediumChunk);
    }
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
    const uint64_t cap_l = g->tuning.light_pair_cap, cap_m = g->tuning.medium_pair_cap;
    const uint32_t force = g->tuning.force_path;
    const uint32_t chunk = g->tuning.heavy_chunk;
    DevMem f1, f2, p1, p2, part;
    DT_TRY(dev_alloc(ctx, f1, (nt + 1) * 8));
    DT_TRY(dev_alloc(ctx, f2, (nt + 1) * 8));
    DT_TRY(dev_alloc(ctx, p1, (nt + 1) * 8));
    DT_TRY(dev_alloc(ctx, p2, (nt + 1) * 8));
    unsigned grid = grid_for(nt, kBlock);
    if (grid > 4096) grid = 4096;
    DT_TRY(dev_alloc(ctx, part, (uint64_t)grid * 5 * 8));
    DT_HIP(hipMemsetAsync(f1.ptr, 0, (nt + 1) * 8, st));
    DT_HIP(hipMemsetAsync(f2.ptr, 0, (nt + 1) * 8, st));
    k_classify<<<grid, kBlock, 0, st>>>(nt, tri.as<uint32_t>(), g->eoff.as<uint32_t>(), cap_l, cap_m, force,
                                        f1.as<uint64_t>(), f2.as<uint64_t>(), part.as<uint64_t>());
    DT_HIP(hipGetLastError());
    std::vector<uint64_t> hp((size_t)grid * 5);
    DT_HIP(hipMemcpyAsync(hp.data(), part.ptr, hp.size() * 8, hipMemcpyDeviceToHost, st));
    DT_TRY(exclusive_scan_u64(ctx, f1.as<uint64_t>(), p1.as<uint64_t>(), nt + 1, st));
    DT_TRY(exclusive_scan_u64(ctx, f2.as<uint64_t>(), p2.as<uint64_t>(), nt + 1, st));
    uint64_t nm = 0, nh = 0;
    DT_HIP(hipMemcpyAsync(&nm, p1.as<uint64_t>() + nt, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipMemcpyAsync(&nh, p2.as<uint64_t>() + nt, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    unsigned __int128 s3 = 0;
    uint64_t bytes = 0, bytes_light = 0, bytes_medium = 0;
    for (unsigned b = 0; b < grid; ++b) {
        s3 += ((unsigned __int128)hp[5 * b + 1] << 64) | hp[5 * b];
        bytes += hp[5 * b + 2];
        bytes_light += hp[5 * b + 3];
        bytes_medium += hp[5 * b + 4];
    }
    g->sum_sigma3 = s3;
    g->alg_bytes = bytes;
    g->alg_bytes_light = bytes_light;
    g->alg_bytes_medium = bytes_medium;
    S.n_heavy = nh;
    S.n_medium = nm;
    S.n_light = nt - nh - nm;
    DT_TRY(dev_alloc(ctx, S.light, S.n_light * 12));
    DT_TRY(dev_alloc(ctx, S.medium, S.n_medium * 12));
    DT_TRY(dev_alloc(ctx, S.heavy, S.n_heavy * 12));
    if (nt) {
        k_partition<<<grid_for(nt, kBlock), kBlock, 0, st>>>(nt, tri.as<uint32_t>(), f1.as<uint64_t>(),
            f2.as<uint64_t>(), p1.as<uint64_t>(), p2.as<uint64_t>(), S.light.as<uint32_t>(),
            S.medium.as<uint32_t>(), S.heavy.as<uint32_t>());
        DT_HIP(hipGetLastError());
    }
    DT_HIP(hipStreamSynchronize(st));
    f1.reset(); f2.reset(); p1.reset(); p2.reset();
    {
        DevMem nch, base;
        DT_TRY(dev_alloc(ctx, nch, (nm + 1) * 8));
        DT_TRY(dev_alloc(ctx, base, (nm + 1) * 8));
        DT_HIP(hipMemsetAsync(nch.ptr, 0, (nm + 1) * 8, st));
        if (nm) {
            k_medium_sizes<<<grid_for(nm, kBlock), kBlock, 0, st>>>(nm, S.medium.as<uint32_t>(),
                                                                    g->eoff.as<uint32_t>(), nch.as<uint64_t>());
            DT_HIP(hipGetLastError());
        }
        DT_TRY(exclusive_scan_u64(ctx, nch.as<uint64_t>(), base.as<uint64_t>(), nm + 1, st));
        uint64_t ni = 0;
        DT_HIP(hipMemcpyAsync(&ni, base.as<uint64_t>() + nm, 8, hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
        S.n_mitems = ni;
        DT_TRY(dev_alloc(ctx, S.mitems, ni * 8));
        if (nm) {
            k_medium_fill<<<grid_for(nm, kBlock), kBlock, 0, st>>>(nm, nch.as<uint64_t>(), base.as<uint64_t>(),
                                                                   S.mitems.as<uint32_t>());
            DT_HIP(hipGetLastError());
        }
        DT_HIP(hipStreamSynchronize(st));
    }
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
