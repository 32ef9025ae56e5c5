// Static triangle enumeration in G_prec (Section 5 and the proof of Theorem 1): for every DAG
// edge (u, v) and every w in N+(u), {u, v, w} is a triangle iff w is also in N+(v); u is then the
// source vertex and u < v < w in the ordering.  The paper tests {v, w} with a hash lookup; here
// one wavefront owns one source vertex u and stages N+(u) (at most degeneracy entries) in LDS.
// For each v in N+(u) the two sorted runs N+(u) after v and N+(v) are intersected by walking the
// shorter and binary-searching the longer (hub vertices late in the ordering have long N+(v)
// runs reached from many u).  The candidates of all v are spread over the 64 lanes through a
// prefix sum of those walk lengths; a hit yields the DAG edge ids of {u, w} and {v, w} directly.
// When the walk over N+(u) is long (kStage entries or more) the longer run N+(v) is first copied
// into LDS, so those searches (most of them on power-law graphs) never touch global memory.
//
// Waves take source vertices from the highest rank down, so the heaviest (the dense core, last in
// the ordering) start first.  Two passes (count per source vertex, exclusive scan, fill) write the
// list in (u, v, w) order with no atomics: triangles sharing a source vertex are adjacent, as are their edge lists in the
// temporal store.  A vertex whose N+(u) exceeds the LDS slice takes the same steps on global memory.
#include "internal.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;
constexpr unsigned kWaves = kBlock / 64;
constexpr uint32_t kCap = 512;    // LDS entries of N+(u) (and of one N+(v)) per wavefront
constexpr uint32_t kStage = 32;   // walks at least this long search an LDS copy of N+(v)
constexpr uint32_t kChunk = 8;    // source vertices taken per grab of the work counter

__device__ __forceinline__ uint32_t find_u32(const uint32_t *a, uint32_t lo, uint32_t hi, uint32_t x) {
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

// position i with pre[i] <= p < pre[i + 1] (pre ascending, pre[0] = 0, du entries)
__device__ __forceinline__ uint32_t owner(const uint32_t *pre, uint32_t du, uint32_t p) {
    uint32_t lo = 0, len = du;
    while (len > 0) {
        uint32_t half = len >> 1;
        if (pre[lo + half] <= p) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo - 1;
}

template <bool FILL>
__global__ void __launch_bounds__(kBlock)
k_tri(uint32_t n, const uint32_t *__restrict__ dag_row, const uint32_t *__restrict__ dag_col,
      uint64_t *__restrict__ cnt, const uint64_t *__restrict__ off, uint32_t *__restrict__ tri,
      unsigned int *__restrict__ next_u, unsigned long long *__restrict__ cand) {
    __shared__ uint32_t s_nbr[kWaves][kCap];
    __shared__ uint32_t s_pre[kWaves][kCap + 1];
    __shared__ uint32_t s_dv[kWaves][kCap];
    __shared__ uint32_t s_vn[kWaves][kCap];
    const unsigned wave = threadIdx.x / 64, lane = threadIdx.x & 63;
    uint32_t *nbr_lds = s_nbr[wave], *pre_lds = s_pre[wave], *dv_lds = s_dv[wave], *vn_lds = s_vn[wave];
    unsigned long long wave_cand = 0;   // candidates of the flattened walks, added once per wave
    for (;;) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(next_u, kChunk);
        base = __shfl(base, 0, 64);
        if (base >= n) break;
        const uint32_t last = base + kChunk < n ? base + kChunk : n;
        // highest rank first: the dense core, with the longest N+ runs, comes last in the ordering
        for (uint32_t ci = base; ci < last; ++ci) {
        const uint32_t u = n - 1 - ci;
        const uint32_t r0 = dag_row[u], du = dag_row[u + 1] - r0;
        uint64_t c = 0;
        uint64_t o = FILL ? off[u] : 0;
        if (du >= 2) {
            const bool in_lds = du <= kCap;
            const uint32_t *nbr = in_lds ? nbr_lds : dag_col + r0;
            // stage N+(u), d+(v) and the prefix of the walk lengths min(du - i - 1, d+(v))
            uint32_t carry = 0;
            for (uint32_t b = 0; b < du; b += 64) {
                const uint32_t i = b + lane;
                uint32_t v = 0, dv = 0;
                if (i < du) {
                    v = dag_col[r0 + i];
                    const uint32_t outv = dag_row[v + 1] - dag_row[v];
                    const uint32_t after = du - i - 1;
                    if (in_lds) {
                        nbr_lds[i] = v;
                        dv_lds[i] = outv;
                    }
                    const bool staged = outv > after && after >= kStage && outv <= kCap;
                    dv = in_lds ? (staged ? 0 : (outv < after ? outv : after)) : (i + 1 < du ? outv : 0);
                }
                uint32_t x = dv;   // inclusive wave scan
#pragma unroll
                for (int s = 1; s < 64; s <<= 1) {
                    uint32_t y = __shfl_up(x, s, 64);
                    if (lane >= (unsigned)s) x += y;
                }
                if (in_lds && i < du) pre_lds[i] = carry + x - dv;
                carry += __shfl(x, 63, 64);
            }
            const uint32_t work = carry;
            wave_cand += work;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            if (in_lds) {
                for (uint32_t b = 0; b < work; b += 64) {
                    const uint32_t p = b + lane;
                    bool hit = false;
                    uint32_t i = 0, j = 0, v = 0, pos = 0;
                    uint32_t e_uw = 0, e_vw = 0;
                    if (p < work) {
                        i = owner(pre_lds, du, p);
                        j = p - pre_lds[i];
                        v = nbr_lds[i];
                        const uint32_t vb = dag_row[v], outv = dv_lds[i];
                        if (outv <= du - i - 1) {
                            // walk N+(v), search N+(u) after v in LDS
                            const uint32_t w = dag_col[vb + j];
                            pos = find_u32(nbr_lds, i + 1, du, w);
                            hit = pos < du && nbr_lds[pos] == w;
                            e_uw = r0 + pos;
                            e_vw = vb + j;
                        } else {
                            // walk N+(u) after v, search N+(v) in global memory
                            const uint32_t w = nbr_lds[i + 1 + j];
                            pos = find_u32(dag_col, vb, vb + outv, w);
                            hit = pos < vb + outv && dag_col[pos] == w;
                            e_uw = r0 + i + 1 + j;
                            e_vw = pos;
                        }
                    }
                    const uint64_t mask = __ballot(hit);
                    if (FILL && hit) {
                        const uint64_t rank = __popcll(mask & ((1ull << lane) - 1));
                        const uint64_t t = o + c + rank;
                        tri[3 * t] = r0 + i;
                        tri[3 * t + 1] = e_uw;
                        tri[3 * t + 2] = e_vw;
                    }
                    c += __popcll(mask);
                }
                // long walks into a long N+(v): copy N+(v) into LDS, then search it there
                for (uint32_t i = 0; i + kStage < du; ++i) {
                    const uint32_t after = du - i - 1, outv = dv_lds[i];
                    if (!(outv > after && after >= kStage && outv <= kCap)) continue;
                    const uint32_t v = nbr_lds[i], vb = dag_row[v];
                    wave_cand += after;
                    __builtin_amdgcn_wave_barrier();
                    for (uint32_t j = lane; j < outv; j += 64) vn_lds[j] = dag_col[vb + j];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __builtin_amdgcn_wave_barrier();
                    for (uint32_t b = 0; b < after; b += 64) {
                        const uint32_t j = b + lane;
                        bool hit = false;
                        uint32_t pos = 0;
                        if (j < after) {
                            const uint32_t w = nbr_lds[i + 1 + j];
                            pos = find_u32(vn_lds, 0, outv, w);
                            hit = pos < outv && vn_lds[pos] == w;
                        }
                        const uint64_t mask = __ballot(hit);
                        if (FILL && hit) {
                            const uint64_t t = o + c + __popcll(mask & ((1ull << lane) - 1));
                            tri[3 * t] = r0 + i;
                            tri[3 * t + 1] = r0 + i + 1 + j;
                            tri[3 * t + 2] = vb + pos;
                        }
                        c += __popcll(mask);
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            } else {
                // N+(u) larger than the LDS slice: the same candidates, v by v, on global memory
                for (uint32_t i = 0; i + 1 < du; ++i) {
                    const uint32_t v = nbr[i];
                    const uint32_t b0 = dag_row[v], dv = dag_row[v + 1] - b0;
                    for (uint32_t b = 0; b < dv; b += 64) {
                        const uint32_t j = b + lane;
                        bool hit = false;
                        uint32_t pos = 0;
                        if (j < dv) {
                            const uint32_t w = dag_col[b0 + j];
                            pos = find_u32(nbr, i + 1, du, w);
                            hit = pos < du && nbr[pos] == w;
                        }
                        const uint64_t mask = __ballot(hit);
                        if (FILL && hit) {
                            const uint64_t t = o + c + __popcll(mask & ((1ull << lane) - 1));
                            tri[3 * t] = r0 + i;
                            tri[3 * t + 1] = r0 + pos;
                            tri[3 * t + 2] = b0 + j;
                        }
                        c += __popcll(mask);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (!FILL && lane == 0) cnt[u] = c;
        }
    }
    if (!FILL && lane == 0) atomicAdd(cand, wave_cand);
}

}  // namespace

int enumerate_triangles(const dt_graph *g, DevMem &tri, uint64_t *ntri_out, uint64_t *cand_out) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    DevMem cnt, off, ctr;
    DT_TRY(dev_alloc(ctx, cnt, ((uint64_t)n + 1) * 8));
    DT_TRY(dev_alloc(ctx, off, ((uint64_t)n + 1) * 8));
    DT_TRY(dev_alloc(ctx, ctr, 256));
    DT_HIP(hipMemsetAsync(cnt.ptr, 0, ((uint64_t)n + 1) * 8, st));
    const unsigned grid = (unsigned)ctx->num_cus * 8;
    if (n) {
        DT_HIP(hipMemsetAsync(ctr.ptr, 0, 4, st));
        DT_HIP(hipMemsetAsync(ctr.as<uint8_t>() + 8, 0, 8, st));
        prof_begin(ctx, kProfTriCount, st);
        k_tri<false><<<grid, kBlock, 0, st>>>(n, g->dag_row.as<uint32_t>(), g->dag_col.as<uint32_t>(),
                                               cnt.as<uint64_t>(), nullptr, nullptr, ctr.as<unsigned>(),
                                               (unsigned long long *)(ctr.as<uint8_t>() + 8));
        prof_end(ctx, kProfTriCount, st);
        DT_HIP(hipGetLastError());
    }
    DT_TRY(exclusive_scan_u64(ctx, cnt.as<uint64_t>(), off.as<uint64_t>(), (uint64_t)n + 1, st));
    uint64_t ntri = 0, cand = 0;
    DT_HIP(hipMemcpyAsync(&ntri, off.as<uint64_t>() + n, 8, hipMemcpyDeviceToHost, st));
    if (n) DT_HIP(hipMemcpyAsync(&cand, ctr.as<uint8_t>() + 8, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    *ntri_out = ntri;
    *cand_out = cand;
    DT_TRY(dev_alloc(ctx, tri, ntri * 12));
    if (n && ntri) {
        DT_HIP(hipMemsetAsync(ctr.ptr, 0, 4, st));
        prof_begin(ctx, kProfTriFill, st);
        k_tri<true><<<grid, kBlock, 0, st>>>(n, g->dag_row.as<uint32_t>(), g->dag_col.as<uint32_t>(),
                                              nullptr, off.as<uint64_t>(), tri.as<uint32_t>(),
                                              ctr.as<unsigned>(), nullptr);
        prof_end(ctx, kProfTriFill, st);
        DT_HIP(hipGetLastError());
    }
    DT_HIP(hipStreamSynchronize(st));
    return DT_OK;
}

}  // namespace dt
