// Count schedule, built once per graph (it does not depend on the deltas, Section 6 "running time
// independent of time periods").  A triangle with one temporal edge per pair becomes a unit record
// (its ordering, orientation and type fixed here, Figures 3 and 4 with Table 2); every other static
// triangle goes to the light path (one lane), the medium path (one wavefront) or the heavy path
// (the prefix-count procedures split over workgroups), decided by P = sigma_uv * sigma_uw, the
// number of (uv edge, uw edge) pairs the pairwise paths walk.  A medium triangle becomes
// ceil(P / kMediumChunk) work items of equal size.  Also the graph totals reported in the
// statistics: the sum over triangles of the product of the three pair multiplicities (the count at
// infinite deltas, an overflow bound) and the algorithmic bytes of one whole-graph count.
#include <algorithm>

#include "count_dev.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;

__device__ __forceinline__ uint32_t ceil_log2_1(uint32_t s) {   // ceil(log2(s + 1))
    return s == 0 ? 0 : 32 - __clz(s);
}

// class 0 light, 1 medium, 2 heavy, 3 unit; force: 0 by the caps, 1 light, 2 heavy, 3 medium
__device__ __forceinline__ int tri_class(uint64_t P, uint64_t cap_l, uint64_t cap_m, uint32_t force,
                                         bool unit) {
    if (force == 0 && unit) return 3;
    if (force == 1) return 0;
    if (force == 2) return 2;
    if (force == 3) return P < (1ull << 31) ? 1 : 2;
    return P <= cap_l ? 0 : (P <= cap_m ? 1 : 2);
}

constexpr int kPartWords = 6;   // per block: sum_sigma3 lo, hi, bytes, light, medium, unit bytes

// per triangle: class flags; per block: the sum of sigma products (128-bit) and the byte totals
__global__ void k_classify(uint64_t n_tri, const uint32_t *__restrict__ tri, const uint32_t *__restrict__ eoff,
                           uint64_t cap_l, uint64_t cap_m, uint32_t force, uint32_t unit_ok,
                           uint64_t *__restrict__ f1, uint64_t *__restrict__ f2, uint64_t *__restrict__ f3,
                           uint64_t *__restrict__ part) {
    __shared__ unsigned long long s_w[kPartWords][kBlock];
    unsigned __int128 acc = 0;
    unsigned long long bytes = 0, bytes_light = 0, bytes_medium = 0, bytes_unit = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n_tri; i += (uint64_t)gridDim.x * kBlock) {
        const uint32_t e_uv = tri[3 * i], e_uw = tri[3 * i + 1], e_vw = tri[3 * i + 2];
        const uint64_t s_uv = eoff[2 * e_uv + 2] - eoff[2 * e_uv];
        const uint64_t s_uw = eoff[2 * e_uw + 2] - eoff[2 * e_uw];
        const uint32_t s_vw = eoff[2 * e_vw + 2] - eoff[2 * e_vw];
        const bool unit = unit_ok && s_uv == 1 && s_uw == 1 && s_vw == 1;
        const int cls = tri_class(s_uv * s_uw, cap_l, cap_m, force, unit);
        f1[i] = cls == 1 ? 1ull : 0ull;
        f2[i] = cls == 2 ? 1ull : 0ull;
        f3[i] = cls == 3 ? 1ull : 0ull;
        acc += (unsigned __int128)(s_uv * s_uw) * s_vw;
        uint64_t b;
        if (cls == 3) {
            b = sizeof(uint4);
        } else {
            const uint32_t probe = 2 * ceil_log2_1(s_vw);
            b = 12 + 36 + 8 * (s_uv + s_uw) + 8 * (uint64_t)(s_vw < probe ? s_vw : probe);
        }
        bytes += b;
        bytes_light += cls == 0 ? b : 0;
        bytes_medium += cls == 1 ? b : 0;
        bytes_unit += cls == 3 ? b : 0;
    }
    s_w[0][threadIdx.x] = (unsigned long long)acc;
    s_w[1][threadIdx.x] = (unsigned long long)(acc >> 64);
    s_w[2][threadIdx.x] = bytes;
    s_w[3][threadIdx.x] = bytes_light;
    s_w[4][threadIdx.x] = bytes_medium;
    s_w[5][threadIdx.x] = bytes_unit;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned __int128 t = 0;
        unsigned long long w[kPartWords] = {0, 0, 0, 0, 0, 0};
        for (unsigned j = 0; j < kBlock; ++j) {
            t += ((unsigned __int128)s_w[1][j] << 64) | s_w[0][j];
            for (int x = 2; x < kPartWords; ++x) w[x] += s_w[x][j];
        }
        part[kPartWords * blockIdx.x] = (uint64_t)t;
        part[kPartWords * blockIdx.x + 1] = (uint64_t)(t >> 64);
        for (int x = 2; x < kPartWords; ++x) part[kPartWords * blockIdx.x + x] = w[x];
    }
}

// The unit record of triangle (e_uv, e_uw, e_vw), each pair holding one temporal edge: the edge's
// key sits at eoff[2e] whichever its direction; the direction bit is 1 (towards the earlier vertex
// of u < v < w) when the pair's forward part [eoff[2e], eoff[2e+1]) is empty.
__device__ __forceinline__ uint4 unit_record(uint32_t e_uv, uint32_t e_uw, uint32_t e_vw,
                                             const uint32_t *__restrict__ eoff,
                                             const uint64_t *__restrict__ key, int shift) {
    const uint32_t es[3] = {e_uv, e_uw, e_vw};
    uint64_t k[3];
    int dir[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const uint32_t a = eoff[2 * es[p]], b = eoff[2 * es[p] + 1];
        k[p] = key[a];
        dir[p] = a == b ? 1 : 0;
    }
    // pairs in key order: first, second, third (0 = uv, 1 = uw, 2 = vw)
    int o0 = 0, o1 = 1, o2 = 2;
    if (k[o1] < k[o0]) { int x = o0; o0 = o1; o1 = x; }
    if (k[o2] < k[o1]) { int x = o1; o1 = o2; o2 = x; }
    if (k[o1] < k[o0]) { int x = o0; o0 = o1; o1 = x; }
    // Figure 3: pi1 (uv, uw, vw), pi2 (uw, uv, vw), pi3 (uv, vw, uw), pi4 (uw, vw, uv),
    // pi5 (vw, uv, uw), pi6 (vw, uw, uv)
    const int pi = o0 == 0 ? (o1 == 1 ? 1 : 3) : (o0 == 1 ? (o1 == 0 ? 2 : 4) : (o1 == 0 ? 5 : 6));
    const int rho = cdev::rho_of(dir[0], dir[1], dir[2]);
    const int type = cdev::psi_of(pi, rho);
    const uint32_t t1 = (uint32_t)(k[o0] >> shift), t2 = (uint32_t)(k[o1] >> shift),
                   t3 = (uint32_t)(k[o2] >> shift);
    return make_uint4(t1, t2 - t1, t3 - t2, (uint32_t)(((pi - 1) * 8 + (rho - 1)) << 8) | (uint32_t)(type - 1));
}

__global__ void k_partition(uint64_t n_tri, const uint32_t *__restrict__ tri, const uint64_t *__restrict__ f1,
                            const uint64_t *__restrict__ f2, const uint64_t *__restrict__ f3,
                            const uint64_t *__restrict__ p1, const uint64_t *__restrict__ p2,
                            const uint64_t *__restrict__ p3, const uint32_t *__restrict__ eoff,
                            const uint64_t *__restrict__ key, int shift, int pos_bits,
                            uint32_t *__restrict__ light,
                            uint32_t *__restrict__ medium, uint32_t *__restrict__ heavy,
                            uint4 *__restrict__ urec, uint64_t *__restrict__ ukey) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_tri) return;
    const uint32_t e_uv = tri[3 * i], e_uw = tri[3 * i + 1], e_vw = tri[3 * i + 2];
    if (f3[i]) {
        // sort key: t1 above the record's position (positions ascend, so the order is stable)
        const uint64_t j = p3[i];
        const uint4 r = unit_record(e_uv, e_uw, e_vw, eoff, key, shift);
        urec[j] = r;
        ukey[j] = ((uint64_t)r.x << pos_bits) | j;
        return;
    }
    uint32_t *dst = f2[i] ? heavy + 3 * p2[i]
                          : (f1[i] ? medium + 3 * p1[i] : light + 3 * (i - p1[i] - p2[i] - p3[i]));
    dst[0] = e_uv;
    dst[1] = e_uw;
    dst[2] = e_vw;
}

// records in t1 order
__global__ void k_unit_gather(uint64_t nu, const uint64_t *__restrict__ skey, uint64_t pos_mask,
                              const uint4 *__restrict__ src, uint4 *__restrict__ dst) {
    uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nu) return;
    dst[j] = src[skey[j] & pos_mask];
}

// t1 of every kUnitStride-th record
__global__ void k_unit_index(uint64_t nidx, const uint4 *__restrict__ rec, uint32_t *__restrict__ idx) {
    uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nidx) return;
    idx[j] = rec[j * kUnitStride].x;
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
    // unit records hold 32-bit relative times and 32-bit positions in their sort key
    const uint32_t unit_ok = g->span <= kUnitMaxSpan && nt < (1ull << 32) ? 1u : 0u;
    DevMem f1, f2, f3, p1, p2, p3, part;
    DT_TRY(dev_alloc(ctx, f1, (nt + 1) * 8));
    DT_TRY(dev_alloc(ctx, f2, (nt + 1) * 8));
    DT_TRY(dev_alloc(ctx, f3, (nt + 1) * 8));
    DT_TRY(dev_alloc(ctx, p1, (nt + 1) * 8));
    DT_TRY(dev_alloc(ctx, p2, (nt + 1) * 8));
    DT_TRY(dev_alloc(ctx, p3, (nt + 1) * 8));
    unsigned grid = grid_for(nt, kBlock);
    if (grid > 4096) grid = 4096;
    DT_TRY(dev_alloc(ctx, part, (uint64_t)grid * kPartWords * 8));
    DT_HIP(hipMemsetAsync(f1.ptr, 0, (nt + 1) * 8, st));
    DT_HIP(hipMemsetAsync(f2.ptr, 0, (nt + 1) * 8, st));
    DT_HIP(hipMemsetAsync(f3.ptr, 0, (nt + 1) * 8, st));
    k_classify<<<grid, kBlock, 0, st>>>(nt, tri.as<uint32_t>(), g->eoff.as<uint32_t>(), cap_l, cap_m, force,
                                        unit_ok, f1.as<uint64_t>(), f2.as<uint64_t>(), f3.as<uint64_t>(),
                                        part.as<uint64_t>());
    DT_HIP(hipGetLastError());
    std::vector<uint64_t> hp((size_t)grid * kPartWords);
    DT_HIP(hipMemcpyAsync(hp.data(), part.ptr, hp.size() * 8, hipMemcpyDeviceToHost, st));
    DT_TRY(exclusive_scan_u64(ctx, f1.as<uint64_t>(), p1.as<uint64_t>(), nt + 1, st));
    DT_TRY(exclusive_scan_u64(ctx, f2.as<uint64_t>(), p2.as<uint64_t>(), nt + 1, st));
    DT_TRY(exclusive_scan_u64(ctx, f3.as<uint64_t>(), p3.as<uint64_t>(), nt + 1, st));
    uint64_t nm = 0, nh = 0, nu = 0;
    DT_HIP(hipMemcpyAsync(&nm, p1.as<uint64_t>() + nt, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipMemcpyAsync(&nh, p2.as<uint64_t>() + nt, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipMemcpyAsync(&nu, p3.as<uint64_t>() + nt, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    unsigned __int128 s3 = 0;
    uint64_t w[kPartWords] = {0, 0, 0, 0, 0, 0};
    for (unsigned b = 0; b < grid; ++b) {
        s3 += ((unsigned __int128)hp[kPartWords * b + 1] << 64) | hp[kPartWords * b];
        for (int x = 2; x < kPartWords; ++x) w[x] += hp[kPartWords * b + x];
    }
    g->sum_sigma3 = s3;
    g->alg_bytes = w[2];
    g->alg_bytes_light = w[3];
    g->alg_bytes_medium = w[4];
    g->alg_bytes_unit = w[5];
    S.n_heavy = nh;
    S.n_medium = nm;
    S.n_unit = nu;
    S.n_light = nt - nh - nm - nu;
    DT_TRY(dev_alloc(ctx, S.light, S.n_light * 12));
    DT_TRY(dev_alloc(ctx, S.medium, S.n_medium * 12));
    DT_TRY(dev_alloc(ctx, S.heavy, S.n_heavy * 12));
    // positions take pos_bits, t1 < 2^31 the bits above: at most 63 in all
    int pos_bits = 0;
    while (pos_bits < 32 && (1ull << pos_bits) < nu) ++pos_bits;
    int t_bits = 0;
    while (t_bits < 31 && (1ll << t_bits) <= g->span) ++t_bits;
    DevMem urec, ukey, skey;
    DT_TRY(dev_alloc(ctx, urec, nu * sizeof(uint4)));
    DT_TRY(dev_alloc(ctx, ukey, nu * 8));
    if (nt) {
        k_partition<<<grid_for(nt, kBlock), kBlock, 0, st>>>(nt, tri.as<uint32_t>(), f1.as<uint64_t>(),
            f2.as<uint64_t>(), f3.as<uint64_t>(), p1.as<uint64_t>(), p2.as<uint64_t>(), p3.as<uint64_t>(),
            g->eoff.as<uint32_t>(), g->key.as<uint64_t>(), g->shift, pos_bits, S.light.as<uint32_t>(),
            S.medium.as<uint32_t>(), S.heavy.as<uint32_t>(), urec.as<uint4>(), ukey.as<uint64_t>());
        DT_HIP(hipGetLastError());
    }
    DT_HIP(hipStreamSynchronize(st));
    f1.reset(); f2.reset(); f3.reset(); p1.reset(); p2.reset(); p3.reset();
    // unit records in t1 order, and the host index of every kUnitStride-th t1
    if (nu) {
        DT_TRY(dev_alloc(ctx, skey, nu * 8));
        DT_TRY(sort_keys_u64(ctx, ukey.as<uint64_t>(), skey.as<uint64_t>(), nu, std::max(1, pos_bits + t_bits), st));
        ukey.reset();
        DT_TRY(dev_alloc(ctx, S.unit, nu * sizeof(uint4)));
        k_unit_gather<<<grid_for(nu, kBlock), kBlock, 0, st>>>(nu, skey.as<uint64_t>(), (1ull << pos_bits) - 1,
                                                               urec.as<uint4>(), S.unit.as<uint4>());
        DT_HIP(hipGetLastError());
        const uint64_t nidx = (nu + kUnitStride - 1) / kUnitStride;
        DevMem didx;
        DT_TRY(dev_alloc(ctx, didx, nidx * 4));
        k_unit_index<<<grid_for(nidx, kBlock), kBlock, 0, st>>>(nidx, S.unit.as<uint4>(), didx.as<uint32_t>());
        DT_HIP(hipGetLastError());
        S.unit_index.resize(nidx);
        DT_HIP(hipMemcpyAsync(S.unit_index.data(), didx.ptr, nidx * 4, hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
    }
    urec.reset();
    skey.reset();
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

void unit_range(const dt_graph *g, const DQuery &q, uint64_t *b, uint64_t *e) {
    const Schedule &S = g->sched;
    *b = 0;
    *e = S.n_unit;
    if (!q.windowed || S.n_unit == 0) return;
    // a triangle inside the window has wlo <= t1 < whi (relative times)
    const uint64_t wlo = q.klo >> q.shift, whi = q.khi >> q.shift;
    const std::vector<uint32_t> &ix = S.unit_index;
    // index entries below wlo: the records before the last of them all have t1 < wlo
    const size_t below = std::lower_bound(ix.begin(), ix.end(), wlo,
                                          [](uint32_t a, uint64_t v) { return (uint64_t)a < v; }) - ix.begin();
    *b = below > 0 ? (uint64_t)(below - 1) * kUnitStride : 0;
    // the first entry at or after whi starts a run of records with t1 >= whi
    const size_t upto = std::lower_bound(ix.begin(), ix.end(), whi,
                                         [](uint32_t a, uint64_t v) { return (uint64_t)a < v; }) - ix.begin();
    if (upto < ix.size()) *e = std::min<uint64_t>((uint64_t)upto * kUnitStride, S.n_unit);
    if (*e < *b) *e = *b;
}

}  // namespace dt
