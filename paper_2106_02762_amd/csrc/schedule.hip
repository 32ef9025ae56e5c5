// Count schedule, built once per graph (it does not depend on the deltas, Section 6 "running time
// independent of time periods").  A triangle with one temporal edge per pair becomes a unit record
// (its ordering, orientation and type fixed here, Figures 3 and 4 with Table 2); every other static
// triangle goes to the light path (one lane), the medium path (one wavefront) or the heavy path
// (the prefix-count procedures split over workgroups), decided by P = sigma_uv * sigma_uw, the
// number of (uv edge, uw edge) pairs the pairwise paths walk.  A medium triangle becomes one entry
// per edge of its smaller source-incident pair.  Unit records are grouped by their first time and
// the light and medium lists by window cell (a necessary condition on the pairs' first and last
// edge times), so that a query with a time window visits only what can fall inside it; the
// results never depend on this order.  Also the graph totals reported in the
// statistics: the sum over triangles of the product of the three pair multiplicities (the count at
// infinite deltas, an overflow bound) and the algorithmic bytes of one whole-graph count.
#include <algorithm>
#include <cstring>

#include "count_dev.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;

__device__ __forceinline__ uint32_t ceil_log2_1(uint32_t s) {   // ceil(log2(s + 1))
    return s == 0 ? 0 : 32 - __clz(s);
}

// class 0 light, 1 medium, 2 heavy, 3 unit; force: 0 by the caps, 1 light, 2 heavy, 3 medium.
// A light lane searches the {v,w} lists once per pair, so a triangle whose {v,w} pair carries more
// than kLightVw edges goes to the medium path, which walks only the pairs within d13.
__device__ __forceinline__ int tri_class(uint64_t P, uint64_t s_vw, uint64_t cap_l, uint64_t cap_m,
                                         uint32_t force, bool unit) {
    if (force == 0 && unit) return 3;
    if (force == 1) return 0;
    if (force == 2) return 2;
    if (force == 3) return P < (1ull << 31) ? 1 : 2;
    return P <= cap_l && s_vw <= cdev::kLightVw ? 0 : (P <= cap_m ? 1 : 2);
}

constexpr int kPartWords = 6;   // per block: sum_sigma3 lo, hi, bytes, light, medium, unit bytes
constexpr unsigned kClsGrid = 4096;   // blocks of the classify and partition passes (grid-stride)

// Per triangle its class (one byte); per block the triangles of each class and the sum of sigma
// products (128-bit) and byte totals.  The partition pass walks the triangles in the same
// block / iteration order, so per-block class counts give every triangle its place.
__global__ void __launch_bounds__(kBlock)
k_classify(uint64_t n_tri, const uint32_t *__restrict__ tri, const uint32_t *__restrict__ eoff,
           uint64_t cap_l, uint64_t cap_m, uint32_t force, uint32_t unit_ok, uint8_t *__restrict__ cls,
           uint32_t *__restrict__ bcnt, uint64_t *__restrict__ part) {
    __shared__ unsigned long long s_w[kPartWords][kBlock / 64];
    __shared__ unsigned s_cnt[4];
    if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    unsigned __int128 acc = 0;
    unsigned long long bytes = 0, bytes_light = 0, bytes_medium = 0, bytes_unit = 0;
    unsigned c[4] = {0, 0, 0, 0};
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n_tri; i += (uint64_t)gridDim.x * kBlock) {
        const uint32_t e_uv = tri[3 * i], e_uw = tri[3 * i + 1], e_vw = tri[3 * i + 2];
        const uint64_t s_uv = eoff[2 * e_uv + 2] - eoff[2 * e_uv];
        const uint64_t s_uw = eoff[2 * e_uw + 2] - eoff[2 * e_uw];
        const uint32_t s_vw = eoff[2 * e_vw + 2] - eoff[2 * e_vw];
        const bool unit = unit_ok && s_uv == 1 && s_uw == 1 && s_vw == 1;
        const int k = tri_class(s_uv * s_uw, s_vw, cap_l, cap_m, force, unit);
        cls[i] = (uint8_t)k;
        c[0] += k == 0;
        c[1] += k == 1;
        c[2] += k == 2;
        c[3] += k == 3;
        acc += (unsigned __int128)(s_uv * s_uw) * s_vw;
        uint64_t b;
        if (k == 3) {
            b = sizeof(uint4);
        } else {
            const uint32_t probe = 2 * ceil_log2_1(s_vw);
            b = 12 + 36 + 8 * (s_uv + s_uw) + 8 * (uint64_t)(s_vw < probe ? s_vw : probe);
        }
        bytes += b;
        bytes_light += k == 0 ? b : 0;
        bytes_medium += k == 1 ? b : 0;
        bytes_unit += k == 3 ? b : 0;
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
        if (c[x]) atomicAdd(&s_cnt[x], c[x]);
    // block sums: within each wavefront by shuffles (the 128-bit sum as two words with carry), then
    // over the wavefronts
    unsigned long long lo = (unsigned long long)acc, hi = (unsigned long long)(acc >> 64);
    unsigned long long w[kPartWords - 2] = {bytes, bytes_light, bytes_medium, bytes_unit};
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long lo2 = __shfl_xor(lo, o, 64), hi2 = __shfl_xor(hi, o, 64);
        const unsigned long long s = lo + lo2;
        hi += hi2 + (s < lo ? 1ull : 0ull);
        lo = s;
#pragma unroll
        for (int x = 0; x < kPartWords - 2; ++x) w[x] += __shfl_xor(w[x], o, 64);
    }
    const unsigned wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        s_w[0][wave] = lo;
        s_w[1][wave] = hi;
        for (int x = 2; x < kPartWords; ++x) s_w[x][wave] = w[x - 2];
    }
    __syncthreads();
    if (threadIdx.x < 4) bcnt[4 * blockIdx.x + threadIdx.x] = s_cnt[threadIdx.x];
    if (threadIdx.x == 0) {
        unsigned __int128 t = 0;
        unsigned long long tw[kPartWords] = {0, 0, 0, 0, 0, 0};
        for (unsigned j = 0; j < kBlock / 64; ++j) {
            t += ((unsigned __int128)s_w[1][j] << 64) | s_w[0][j];
            for (int x = 2; x < kPartWords; ++x) tw[x] += s_w[x][j];
        }
        part[kPartWords * blockIdx.x] = (uint64_t)t;
        part[kPartWords * blockIdx.x + 1] = (uint64_t)(t >> 64);
        for (int x = 2; x < kPartWords; ++x) part[kPartWords * blockIdx.x + x] = tw[x];
    }
}

// One workgroup: every classify block's first position in each class list (base, [block][class])
// and the totals: tot[0..3] class sizes, tot[4..5] the 128-bit sum of sigma products, tot[6..9]
// the byte totals.
__global__ void __launch_bounds__(kBlock)
k_cls_totals(unsigned nblk, const uint32_t *__restrict__ bcnt, const uint64_t *__restrict__ part,
             uint64_t *__restrict__ base, uint64_t *__restrict__ tot) {
    __shared__ unsigned long long s_tot[kBlock];
    const unsigned tid = threadIdx.x;
    const unsigned per = (nblk + kBlock - 1) / kBlock;
    const unsigned b0 = min(tid * per, nblk), b1 = min(b0 + per, nblk);
    for (int c = 0; c < 4; ++c) {
        unsigned long long mine = 0;
        for (unsigned b = b0; b < b1; ++b) mine += bcnt[4 * b + c];
        s_tot[tid] = mine;
        __syncthreads();
        // exclusive prefix over threads (Hillis-Steele on the LDS copy)
        for (unsigned o = 1; o < kBlock; o <<= 1) {
            const unsigned long long y = tid >= o ? s_tot[tid - o] : 0ull;
            __syncthreads();
            s_tot[tid] += y;
            __syncthreads();
        }
        unsigned long long run = s_tot[tid] - mine;
        for (unsigned b = b0; b < b1; ++b) {
            base[4 * b + c] = run;
            run += bcnt[4 * b + c];
        }
        if (tid == kBlock - 1) tot[c] = s_tot[tid];
        __syncthreads();
    }
    // the sums of the blocks' partial words, each thread over its blocks, then by shuffles
    unsigned __int128 t = 0;
    unsigned long long w[kPartWords] = {0, 0, 0, 0, 0, 0};
    for (unsigned b = b0; b < b1; ++b) {
        t += ((unsigned __int128)part[kPartWords * b + 1] << 64) | part[kPartWords * b];
        for (int x = 2; x < kPartWords; ++x) w[x] += part[kPartWords * b + x];
    }
    unsigned long long lo = (unsigned long long)t, hi = (unsigned long long)(t >> 64);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long lo2 = __shfl_xor(lo, o, 64), hi2 = __shfl_xor(hi, o, 64);
        const unsigned long long sum = lo + lo2;
        hi += hi2 + (sum < lo ? 1ull : 0ull);
        lo = sum;
#pragma unroll
        for (int x = 2; x < kPartWords; ++x) w[x] += __shfl_xor(w[x], o, 64);
    }
    __shared__ unsigned long long s_part[kBlock / 64][kPartWords];
    if ((tid & 63) == 0) {
        s_part[tid / 64][0] = lo;
        s_part[tid / 64][1] = hi;
        for (int x = 2; x < kPartWords; ++x) s_part[tid / 64][x] = w[x];
    }
    __syncthreads();
    if (tid == 0) {
        unsigned __int128 tt = 0;
        unsigned long long tw[kPartWords] = {0, 0, 0, 0, 0, 0};
        for (unsigned j = 0; j < kBlock / 64; ++j) {
            tt += ((unsigned __int128)s_part[j][1] << 64) | s_part[j][0];
            for (int x = 2; x < kPartWords; ++x) tw[x] += s_part[j][x];
        }
        tot[4] = (uint64_t)tt;
        tot[5] = (uint64_t)(tt >> 64);
        for (int x = 2; x < kPartWords; ++x) tot[4 + x] = tw[x];
    }
}

// Window cell of a light or medium triangle: slice of F (the latest first-edge time over its three
// pairs) times kSlices plus slice of L (the earliest last-edge time).  Each pair's two direction
// lists are key-sorted, so its first and last edges are at their ends.
__device__ __forceinline__ uint16_t window_cell(uint32_t e_uv, uint32_t e_uw, uint32_t e_vw,
                                                const uint32_t *__restrict__ eoff,
                                                const uint64_t *__restrict__ key, int shift, int cshift) {
    const uint32_t es[3] = {e_uv, e_uw, e_vw};
    uint64_t F = 0, L = ~0ull;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const uint32_t a = eoff[2 * es[p]], b = eoff[2 * es[p] + 1], c = eoff[2 * es[p] + 2];
        uint64_t first = ~0ull, last = 0;
        if (a < b) {
            first = key[a];
            last = key[b - 1];
        }
        if (b < c) {
            first = key[b] < first ? key[b] : first;
            last = key[c - 1] > last ? key[c - 1] : last;
        }
        F = first > F ? first : F;
        L = last < L ? last : L;
    }
    const uint64_t f = (F >> shift) >> cshift, l = (L >> shift) >> cshift;
    return (uint16_t)((f < kSlices - 1 ? f : kSlices - 1) * kSlices + (l < kSlices - 1 ? l : kSlices - 1));
}

// Every triangle to its class's list at base[class][block] + its rank in the block's walk; unit
// triangles become records (in triangle order) with their t1 bucket as a sort key; light and
// medium triangles also go, with their window cell as a sort key, to the windowed copies.
__global__ void __launch_bounds__(kBlock)
k_partition(uint64_t n_tri, const uint32_t *__restrict__ tri, const uint8_t *__restrict__ cls,
            const uint64_t *__restrict__ base, const uint32_t *__restrict__ eoff,
            const uint64_t *__restrict__ key, int shift, int bshift, int cshift, uint32_t *__restrict__ light,
            uint32_t *__restrict__ medium, uint32_t *__restrict__ heavy, uint4 *__restrict__ lrec,
            uint16_t *__restrict__ lkey, uint4 *__restrict__ mrec, uint16_t *__restrict__ mkey,
            uint4 *__restrict__ urec, uint16_t *__restrict__ ubkt) {
    __shared__ unsigned long long s_wave[kBlock / 64];
    const unsigned lane = threadIdx.x & 63, wave = threadIdx.x / 64;
    uint64_t run[4] = {base[4 * blockIdx.x], base[4 * blockIdx.x + 1], base[4 * blockIdx.x + 2],
                       base[4 * blockIdx.x + 3]};
    for (uint64_t b0 = (uint64_t)blockIdx.x * kBlock; b0 < n_tri; b0 += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i = b0 + threadIdx.x;
        const int k = i < n_tri ? cls[i] : 4;
        // four 16-bit class counters in one word (a block holds at most 256 triangles)
        const unsigned long long f = k < 4 ? 1ull << (16 * k) : 0ull;
        unsigned long long x = f;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long y = __shfl_up(x, o, 64);
            if (lane >= (unsigned)o) x += y;
        }
        if (lane == 63) s_wave[wave] = x;
        __syncthreads();
        unsigned long long before = 0, total = 0;
#pragma unroll
        for (unsigned w = 0; w < kBlock / 64; ++w) {
            before += w < wave ? s_wave[w] : 0ull;
            total += s_wave[w];
        }
        __syncthreads();
        if (k < 4) {
            const uint64_t pos = run[k] + (((before + x - f) >> (16 * k)) & 0xffffull);
            const uint32_t e_uv = tri[3 * i], e_uw = tri[3 * i + 1], e_vw = tri[3 * i + 2];
            if (k == 3) {
                const uint4 r = cdev::unit_record(e_uv, e_uw, e_vw, eoff, key, shift);
                urec[pos] = r;
                ubkt[pos] = (uint16_t)(r.x >> bshift);
            } else {
                uint32_t *dst = (k == 0 ? light : (k == 1 ? medium : heavy)) + 3 * pos;
                dst[0] = e_uv;
                dst[1] = e_uw;
                dst[2] = e_vw;
                if (k < 2) {
                    (k == 0 ? lrec : mrec)[pos] = make_uint4(e_uv, e_uw, e_vw, 0u);
                    (k == 0 ? lkey : mkey)[pos] = window_cell(e_uv, e_uw, e_vw, eoff, key, shift, cshift);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) run[c] += (total >> (16 * c)) & 0xffffull;
    }
}

// bucket starts from the sorted bucket keys: start[x] for every x in (key[j - 1], key[j]] is j;
// j = nu closes the array at nbk
__global__ void k_unit_starts(uint64_t nu, uint32_t nbk, const uint16_t *__restrict__ bkt,
                              uint32_t *__restrict__ start) {
    uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j > nu) return;
    const int64_t cur = j < nu ? (int64_t)bkt[j] : (int64_t)nbk;
    const int64_t prev = j > 0 ? (int64_t)bkt[j - 1] : -1;
    for (int64_t x = prev + 1; x <= cur; ++x) start[x] = (uint32_t)j;
}

// first position of every cell in a cell-sorted key array (kCells + 1 entries, the last = n)
__global__ void k_cell_starts(uint64_t n, const uint16_t *__restrict__ ck, uint64_t *__restrict__ start) {
    uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j > n) return;
    const int64_t cur = j < n ? (int64_t)ck[j] : (int64_t)kCells;
    const int64_t prev = j > 0 ? (int64_t)ck[j - 1] : -1;
    for (int64_t x = prev + 1; x <= cur; ++x) start[x] = j;
}

// (e_uv, e_uw, e_vw, -) records back to three words per triangle
__global__ void k_unpack3(uint64_t n, const uint4 *__restrict__ rec, uint32_t *__restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint4 r = rec[i];
    out[3 * i] = r.x;
    out[3 * i + 1] = r.y;
    out[3 * i + 2] = r.z;
}

// first medium item of every cell: the item base of the cell's first triangle
__global__ void k_cell_items(const uint64_t *__restrict__ tstart, const uint64_t *__restrict__ ibase,
                             uint64_t *__restrict__ istart) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c <= kCells) istart[c] = ibase[tstart[c]];
}

// entries of the medium path: one per edge of the outer pair (the source-incident pair with fewer
// temporal edges)
__global__ void k_medium_sizes(uint64_t nm, const uint32_t *__restrict__ med, const uint32_t *__restrict__ eoff,
                               uint64_t *__restrict__ nch) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nm) return;
    const uint32_t e_uv = med[3 * i], e_uw = med[3 * i + 1];
    const uint32_t s_uv = eoff[2 * e_uv + 2] - eoff[2 * e_uv], s_uw = eoff[2 * e_uw + 2] - eoff[2 * e_uw];
    nch[i] = cdev::medium_outer_is_uv(s_uv, s_uw) ? s_uv : s_uw;
}

__global__ void k_medium_fill(uint64_t nm, const uint64_t *__restrict__ nch, const uint64_t *__restrict__ base,
                              uint32_t *__restrict__ items) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nm) return;
    for (uint64_t j = 0; j < nch[i]; ++j) {
        items[2 * (base[i] + j)] = (uint32_t)i;
        items[2 * (base[i] + j) + 1] = (uint32_t)j;
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

// Sort n (cell, record) pairs by cell, unpack the records to out (three words per triangle) and
// write the cell starts (kCells + 1 entries) to start.
int cell_order(dt_ctx *ctx, uint64_t n, DevMem &ckey, DevMem &rec, DevMem &out, DevMem &start, hipStream_t st) {
    DevMem k2, r2;
    DT_TRY(dev_alloc(ctx, start, (uint64_t)(kCells + 1) * 8));
    DT_TRY(dev_alloc(ctx, k2, n * 2));
    DT_TRY(dev_alloc(ctx, r2, n * sizeof(uint4)));
    DT_TRY(sort_pairs_u16_u4(ctx, ckey.as<uint16_t>(), k2.as<uint16_t>(), rec.as<uint4>(), r2.as<uint4>(), n, 16, st));
    k_cell_starts<<<grid_for(n + 1, kBlock), kBlock, 0, st>>>(n, k2.as<uint16_t>(), start.as<uint64_t>());
    DT_HIP(hipGetLastError());
    if (n) {
        k_unpack3<<<grid_for(n, kBlock), kBlock, 0, st>>>(n, r2.as<uint4>(), out.as<uint32_t>());
        DT_HIP(hipGetLastError());
    }
    return DT_OK;
}

// Work items of the medium list med (nm triangles): medium_sizes enqueues each triangle's item
// count (nch) and first item (base, nm + 1 entries) and the total's read-back to *total (pinned
// host memory, valid after the stream is synchronised); medium_fill then writes the items.
int medium_sizes(dt_ctx *ctx, uint64_t nm, DevMem &med, DevMem &eoff, DevMem &nch, DevMem &base, uint64_t *total,
                 hipStream_t st) {
    DT_TRY(dev_alloc(ctx, nch, (nm + 1) * 8));
    DT_TRY(dev_alloc(ctx, base, (nm + 1) * 8));
    DT_HIP(hipMemsetAsync(nch.ptr, 0, (nm + 1) * 8, st));
    if (nm) {
        k_medium_sizes<<<grid_for(nm, kBlock), kBlock, 0, st>>>(nm, med.as<uint32_t>(), eoff.as<uint32_t>(),
                                                                nch.as<uint64_t>());
        DT_HIP(hipGetLastError());
    }
    DT_TRY(exclusive_scan_u64(ctx, nch.as<uint64_t>(), base.as<uint64_t>(), nm + 1, st));
    DT_HIP(hipMemcpyAsync(total, base.as<uint64_t>() + nm, 8, hipMemcpyDeviceToHost, st));
    return DT_OK;
}

int medium_fill(dt_ctx *ctx, uint64_t nm, DevMem &nch, DevMem &base, uint64_t ni, DevMem &items, hipStream_t st) {
    DT_TRY(dev_alloc(ctx, items, ni * 8));
    if (nm) {
        k_medium_fill<<<grid_for(nm, kBlock), kBlock, 0, st>>>(nm, nch.as<uint64_t>(), base.as<uint64_t>(),
                                                               items.as<uint32_t>());
        DT_HIP(hipGetLastError());
    }
    return DT_OK;
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
    // unit records hold 32-bit relative times
    const uint32_t unit_ok = g->span <= kUnitMaxSpan ? 1u : 0u;
    const unsigned grid = kClsGrid;
    DevMem cls, bcnt, part, base;
    DT_TRY(dev_alloc(ctx, cls, nt + 1));
    DT_TRY(dev_alloc(ctx, bcnt, (uint64_t)grid * 4 * 4));
    DT_TRY(dev_alloc(ctx, part, (uint64_t)grid * kPartWords * 8));
    DT_TRY(dev_alloc(ctx, base, (uint64_t)grid * 4 * 8));
    k_classify<<<grid, kBlock, 0, st>>>(nt, tri.as<uint32_t>(), g->eoff.as<uint32_t>(), cap_l, cap_m, force,
                                        unit_ok, cls.as<uint8_t>(), bcnt.as<uint32_t>(), part.as<uint64_t>());
    DT_HIP(hipGetLastError());
    DevMem tot;
    DT_TRY(dev_alloc(ctx, tot, 16 * 8));
    k_cls_totals<<<1, kBlock, 0, st>>>(grid, bcnt.as<uint32_t>(), part.as<uint64_t>(), base.as<uint64_t>(),
                                       tot.as<uint64_t>());
    DT_HIP(hipGetLastError());
    uint64_t *hs = reinterpret_cast<uint64_t *>(ctx->pinned_stage);
    DT_HIP(hipMemcpyAsync(hs, tot.ptr, 10 * 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    uint64_t ncls[4] = {hs[0], hs[1], hs[2], hs[3]};
    const unsigned __int128 s3 = ((unsigned __int128)hs[5] << 64) | hs[4];
    const uint64_t w[kPartWords] = {0, 0, hs[6], hs[7], hs[8], hs[9]};
    g->sum_sigma3 = s3;
    g->alg_bytes = w[2];
    g->alg_bytes_light = w[3];
    g->alg_bytes_medium = w[4];
    g->alg_bytes_unit = w[5];
    const uint64_t nm = ncls[1], nh = ncls[2], nu = ncls[3];
    if (ncls[0] + nm + nh + nu != nt) return fail(DT_EDEVICE, "triangle classes do not add up");
    S.n_light = ncls[0];
    S.n_medium = nm;
    S.n_heavy = nh;
    S.n_unit = nu;
    DT_TRY(dev_alloc(ctx, S.light, S.n_light * 12));
    DT_TRY(dev_alloc(ctx, S.medium, S.n_medium * 12));
    DT_TRY(dev_alloc(ctx, S.heavy, S.n_heavy * 12));
    // t1 buckets of the unit records: at most 2^16, t1 >> unit_shift
    int t_bits = 0;
    while (t_bits < 31 && (1ll << t_bits) <= g->span) ++t_bits;
    S.unit_shift = t_bits > 16 ? t_bits - 16 : 0;
    const uint64_t nbk = unit_ok ? ((uint64_t)g->span >> S.unit_shift) + 1 : 1;
    // time slices of the window index: span >> cell_shift < kSlices
    S.cell_shift = 0;
    while (S.cell_shift < 62 && (g->span >> S.cell_shift) >= (int64_t)kSlices) ++S.cell_shift;
    DevMem urec, ubkt, ubkt2, ustart, lrec, lkey, mrec, mkey, lstart, mstart;
    DT_TRY(dev_alloc(ctx, urec, nu * sizeof(uint4)));
    DT_TRY(dev_alloc(ctx, ubkt, nu * 2));
    DT_TRY(dev_alloc(ctx, lrec, S.n_light * sizeof(uint4)));
    DT_TRY(dev_alloc(ctx, lkey, S.n_light * 2));
    DT_TRY(dev_alloc(ctx, mrec, nm * sizeof(uint4)));
    DT_TRY(dev_alloc(ctx, mkey, nm * 2));
    if (nt) {
        k_partition<<<grid, kBlock, 0, st>>>(nt, tri.as<uint32_t>(), cls.as<uint8_t>(), base.as<uint64_t>(),
            g->eoff.as<uint32_t>(), g->key.as<uint64_t>(), g->shift, S.unit_shift, S.cell_shift,
            S.light.as<uint32_t>(), S.medium.as<uint32_t>(), S.heavy.as<uint32_t>(), lrec.as<uint4>(),
            lkey.as<uint16_t>(), mrec.as<uint4>(), mkey.as<uint16_t>(), urec.as<uint4>(), ubkt.as<uint16_t>());
        DT_HIP(hipGetLastError());
    }
    cls.reset();
    // unit records ordered by t1 bucket (a stable two-pass radix sort on the 16-bit bucket) on the
    // first side stream, while this stream builds the other lists; the host keeps the bucket starts
    // (read back through the pinned staging buffer from byte kStageUnit; the light cell starts and
    // the other read-backs use the words before it)
    constexpr size_t kStageUnit = 16384;
    static_assert((kCells + 1) * 8 <= kStageUnit, "staging layout");
    if (kStageUnit + (nbk + 1) * 4 > kPinnedStage) return fail(DT_EDEVICE, "unit bucket index exceeds staging");
    DevMem usort_tmp;
    const hipStream_t us = nu && ctx->side[0] ? ctx->side[0] : st;
    // an early return must not release buffers the side stream still uses
    struct Join {
        hipStream_t s, main;
        ~Join() {
            if (s != main) (void)hipStreamSynchronize(s);
        }
    } join{us, st};
    if (nu) {
        DT_TRY(dev_alloc(ctx, ubkt2, nu * 2));
        DT_TRY(dev_alloc(ctx, S.unit, nu * sizeof(uint4)));
        DT_TRY(dev_alloc(ctx, ustart, (nbk + 1) * 4));
        if (us != st) {
            DT_HIP(hipEventRecord(ctx->ev_relay[0], st));
            DT_HIP(hipStreamWaitEvent(us, ctx->ev_relay[0], 0));
        }
        DT_TRY(sort_pairs_u16_u4(ctx, ubkt.as<uint16_t>(), ubkt2.as<uint16_t>(), urec.as<uint4>(), S.unit.as<uint4>(),
                                 nu, 16, us, us != st ? &usort_tmp : nullptr));
        k_unit_starts<<<grid_for(nu + 1, kBlock), kBlock, 0, us>>>(nu, (uint32_t)nbk, ubkt2.as<uint16_t>(),
                                                                   ustart.as<uint32_t>());
        DT_HIP(hipGetLastError());
        S.unit_index.resize(nbk + 1);
        DT_HIP(hipMemcpyAsync(ctx->pinned_stage + kStageUnit, ustart.ptr, (nbk + 1) * 4, hipMemcpyDeviceToHost, us));
        if (us != st) DT_HIP(hipEventRecord(ctx->ev_relay[1], us));
    }
    // the windowed copies of the light and medium lists, in window-cell order
    DT_TRY(dev_alloc(ctx, S.light_w, S.n_light * 12));
    DT_TRY(dev_alloc(ctx, S.medium_w, nm * 12));
    DT_TRY(cell_order(ctx, S.n_light, lkey, lrec, S.light_w, lstart, st));
    DT_TRY(cell_order(ctx, nm, mkey, mrec, S.medium_w, mstart, st));
    S.light_cells.resize(kCells + 1);
    DT_HIP(hipMemcpyAsync(ctx->pinned_stage, lstart.ptr, (kCells + 1) * 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    memcpy(S.light_cells.data(), ctx->pinned_stage, (kCells + 1) * 8);
    // medium work items of both copies (the same totals: the same triangles in another order)
    {
        DevMem nch0, base0, nch1, base;
        uint64_t *ni2 = reinterpret_cast<uint64_t *>(ctx->pinned_stage);
        DT_TRY(medium_sizes(ctx, nm, S.medium, g->eoff, nch0, base0, &ni2[0], st));
        DT_TRY(medium_sizes(ctx, nm, S.medium_w, g->eoff, nch1, base, &ni2[1], st));
        DT_HIP(hipStreamSynchronize(st));
        const uint64_t ni = ni2[0], ni_w = ni2[1];
        if (ni != ni_w) return fail(DT_EDEVICE, "medium work items of the two orders differ");
        DT_TRY(medium_fill(ctx, nm, nch0, base0, ni, S.mitems, st));
        DT_TRY(medium_fill(ctx, nm, nch1, base, ni_w, S.mitems_w, st));
        S.n_mitems = ni;
        DevMem istart;
        DT_TRY(dev_alloc(ctx, istart, (uint64_t)(kCells + 1) * 8));
        k_cell_items<<<grid_for(kCells + 1, kBlock), kBlock, 0, st>>>(mstart.as<uint64_t>(), base.as<uint64_t>(),
                                                                      istart.as<uint64_t>());
        DT_HIP(hipGetLastError());
        S.mitem_cells.resize(kCells + 1);
        DT_HIP(hipMemcpyAsync(ctx->pinned_stage, istart.ptr, (kCells + 1) * 8, hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
        memcpy(S.mitem_cells.data(), ctx->pinned_stage, (kCells + 1) * 8);
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
    uint64_t *htot = reinterpret_cast<uint64_t *>(ctx->pinned_stage);
    DT_HIP(hipMemcpyAsync(&htot[0], S.hslot.as<uint64_t>() + nh, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipMemcpyAsync(&htot[1], cbase.as<uint64_t>() + nh, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    S.n_slots = htot[0];
    S.n_chunks = htot[1];
    if (S.n_chunks > 0xffffffffull || nh > 0xffffffffull)
        return fail(DT_EOVERFLOW, "too many heavy work items (%llu)", (unsigned long long)S.n_chunks);
    DT_TRY(dev_alloc(ctx, S.chunks, S.n_chunks * 8));
    if (nh) {
        k_heavy_chunks<<<grid_for(nh, kBlock), kBlock, 0, st>>>(nh, nch.as<uint64_t>(), cbase.as<uint64_t>(),
                                                                chunk, S.chunks.as<uint32_t>());
        DT_HIP(hipGetLastError());
    }
    // join the unit-record sort
    if (nu && us != st) DT_HIP(hipStreamWaitEvent(st, ctx->ev_relay[1], 0));
    DT_HIP(hipStreamSynchronize(st));
    if (nu) memcpy(S.unit_index.data(), ctx->pinned_stage + kStageUnit, (nbk + 1) * 4);
    return DT_OK;
}

void cell_ranges(const std::vector<uint64_t> &ix, int cell_shift, const DQuery &q, Ranges &r) {
    r.n = 0;
    r.pre[0] = 0;
    if (ix.size() != kCells + 1 || ix[kCells] == 0) return;
    auto add = [&](uint64_t b, uint64_t e) {
        if (e <= b) return;
        if (r.n && r.b[r.n - 1] + (r.pre[r.n] - r.pre[r.n - 1]) == b) {
            r.pre[r.n] += e - b;   // adjacent to the previous range
            return;
        }
        r.b[r.n] = b;
        r.pre[r.n + 1] = r.pre[r.n] + (e - b);
        ++r.n;
    };
    if (!q.windowed) {
        add(0, ix[kCells]);
        return;
    }
    // relative times [wlo, whi) of the window; cells (f, l) with f <= slice(whi - 1), l >= slice(wlo)
    const uint64_t wlo = q.klo >> q.shift, whi = q.khi >> q.shift;
    if (whi <= wlo) return;
    const uint64_t ql = std::min<uint64_t>(wlo >> cell_shift, kSlices - 1);
    const uint64_t qh = std::min<uint64_t>((whi - 1) >> cell_shift, kSlices - 1);
    for (uint64_t f = 0; f <= qh; ++f) add(ix[f * kSlices + ql], ix[f * kSlices + kSlices]);
}

void unit_range(const dt_graph *g, const DQuery &q, uint64_t *b, uint64_t *e) {
    const Schedule &S = g->sched;
    *b = 0;
    *e = S.n_unit;
    if (!q.windowed || S.n_unit == 0) return;
    // a triangle inside the window has wlo <= t1 < whi (relative times): buckets
    // wlo >> shift .. (whi - 1) >> shift
    const std::vector<uint32_t> &ix = S.unit_index;   // bucket starts, nbk + 1 entries
    const uint64_t nbk = ix.size() - 1;
    const uint64_t wlo = q.klo >> q.shift, whi = q.khi >> q.shift;
    if (whi <= wlo) {
        *e = *b;
        return;
    }
    const uint64_t bl = std::min<uint64_t>(wlo >> S.unit_shift, nbk);
    const uint64_t bh = std::min<uint64_t>(((whi - 1) >> S.unit_shift) + 1, nbk);
    *b = ix[bl];
    *e = bh > bl ? ix[bh] : ix[bl];
}

}  // namespace dt
