// Count schedule, built once per graph (it does not depend on the deltas, Section 6 "running time
// independent of time periods").  A triangle with one temporal edge per pair becomes a unit record
// (its ordering, orientation and type fixed here, Figures 3 and 4 with Table 2); a triangle with
// few (uv edge, uw edge) pairs goes to the light path (one lane).  Every other triangle is split
// between the medium path, whose work is the number of close pairs (growing with d13), and the
// prefix-count procedures of Algorithms 1-3 (work (sigma_uv + sigma_uw) log sigma, Theorem 1) by a
// cost model: its pair budget is the prefix procedures' cost over the medium path's cost per pair.
// A triangle whose P = sigma_uv sigma_uw pairs fit the budget is always medium; one whose outer
// edges alone exceed it is always heavy; for the others (contested) a wavefront finds the largest
// level l such that its pairs within D(l) = 2^(l-1) - 1 of each other fit, by binary search over
// the levels with exact close-pair counts.  Contested triangles are sorted by descending level, so
// that a whole-span query walks a prefix of the medium list and a suffix of the heavy list.  A
// medium triangle becomes one entry per edge of its smaller source-incident pair (times the chunks
// of its other one, when that one is long and the triangle not too large); a heavy one gets
// count chunks of 256 source edges and prefix chunks of 256 edges of one list.  Unit records are
// grouped by their first time and the light and medium lists copied in window-cell order (a
// necessary condition on the pairs' first and last edge times), so that a query with a time
// window visits only what can fall inside it; the results never depend on any of these orders.
// Also the graph totals reported in the statistics: the sum over triangles of the product of the
// three pair multiplicities (the count at infinite deltas, an overflow bound) and the algorithmic
// bytes of one whole-graph count.
#include <algorithm>
#include <cstring>

#include "count_dev.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;

__device__ __forceinline__ uint32_t ceil_log2_1(uint32_t s) {   // ceil(log2(s + 1))
    return s == 0 ? 0 : 32 - __clz(s);
}

enum : int { kClsLight = 0, kClsMedium = 1, kClsHeavy = 2, kClsUnit = 3, kClsContest = 4 };
constexpr int kClasses = 5;
// the medium path's per-lane counts are 32-bit sums over a wavefront: inner pairs stay below 2^25
constexpr uint64_t kMediumMaxInner = 1ull << 25;
constexpr uint32_t kCrossSample = 128;   // outer edges sampled by the level search

struct SplitRule {
    uint64_t cap_l, cap_m;
    uint32_t force, unit_ok, cost_pct;
};

// The pair budget of a triangle outside the light rule: how many (uv edge, uw edge) pairs the
// medium path may evaluate before its cost passes the prefix procedures' cost times cost_pct / 100.
// Costs are counted in binary-search steps of the searches each path makes: the medium path pays 4
// searches into the inner source pair (or into each chunk of it) per outer edge plus a fixed
// overhead, then about 10 searches into the {v,w} lists per close pair; the prefix procedures pay per source edge 14 searches into
// the other source pair and 24 into the {v,w} lists (prefix and count passes) plus an overhead.
__device__ __forceinline__ double pair_budget(uint64_t s_uv, uint64_t s_uw, uint64_t s_vw, uint32_t cost_pct) {
    const double luv = ceil_log2_1((uint32_t)s_uv) + 1.0, luw = ceil_log2_1((uint32_t)s_uw) + 1.0,
                 lvw = ceil_log2_1((uint32_t)s_vw) + 1.0;
    const double heavy = (double)s_uv * (14.0 * luw + 24.0 * lvw + 12.0) + (double)s_uw * (14.0 * luv + 24.0 * lvw + 12.0);
    const bool outer_uv = cdev::medium_outer_is_uv((uint32_t)s_uv, (uint32_t)s_uw);
    const uint32_t chunks = cdev::medium_inner_chunks((uint32_t)(outer_uv ? s_uv : s_uw), (uint32_t)(outer_uv ? s_uw : s_uv));
    const double lin = chunks > 1 ? ceil_log2_1(cdev::kInnerChunk) + 1.0 : (outer_uv ? luw : luv);
    const double outer = (double)(outer_uv ? s_uv : s_uw) * chunks * (4.0 * lin + 8.0);
    return (heavy * cost_pct / 100.0 - outer) / (10.0 * lvw + 6.0);
}

// class of a triangle: unit, light, always medium, always heavy, or contested
__device__ __forceinline__ int tri_class(uint64_t s_uv, uint64_t s_uw, uint64_t s_vw, const SplitRule &R) {
    const uint64_t P = s_uv * s_uw;
    if (R.force == 0 && R.unit_ok && s_uv == 1 && s_uw == 1 && s_vw == 1) return kClsUnit;
    if (R.force == 1) return kClsLight;
    if (R.force == 2) return kClsHeavy;
    if (R.force == 3) return P < (1ull << 31) && s_uv < kMediumMaxInner && s_uw < kMediumMaxInner ? kClsMedium : kClsHeavy;
    if (P <= R.cap_l && s_vw <= cdev::kLightVw) return kClsLight;
    if (P > R.cap_m || s_uv >= kMediumMaxInner || s_uw >= kMediumMaxInner) return kClsHeavy;
    const double B = pair_budget(s_uv, s_uw, s_vw, R.cost_pct);
    if (B < 0.0) return kClsHeavy;
    if ((double)P <= B) return kClsMedium;
    return kClsContest;
}

constexpr int kPartWords = 6;   // per block: sum_sigma3 lo, hi, bytes, light, medium, unit bytes
constexpr unsigned kClsGrid = 4096;   // blocks of the classify and partition passes (grid-stride)
constexpr int kTotWords = kClasses + kPartWords;   // class sizes, then the partial words

// Per list entry its class (one byte; kClasses for an empty entry); per block the triangles of
// each class and the sum of sigma products (128-bit) and byte totals.  The partition pass walks the
// entries in the same block / iteration order, so per-block class counts give every triangle its
// place.
__global__ void __launch_bounds__(kBlock)
k_classify(uint64_t n_tri, const uint32_t *__restrict__ tri, const uint32_t *__restrict__ eoff, SplitRule R,
           uint8_t *__restrict__ cls, uint32_t *__restrict__ bcnt, uint64_t *__restrict__ part) {
    __shared__ unsigned long long s_w[kPartWords][kBlock / 64];
    __shared__ unsigned s_cnt[kClasses];
    if (threadIdx.x < kClasses) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    unsigned __int128 acc = 0;
    unsigned long long bytes = 0, bytes_light = 0, bytes_medium = 0, bytes_unit = 0;
    unsigned c[kClasses] = {0, 0, 0, 0, 0};
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n_tri; i += (uint64_t)gridDim.x * kBlock) {
        const uint32_t e_uv = tri[3 * i], e_uw = tri[3 * i + 1], e_vw = tri[3 * i + 2];
        if (e_uv == kNoEdge) {   // an empty entry: no class
            cls[i] = (uint8_t)kClasses;
            continue;
        }
        const uint64_t s_uv = eoff[2 * e_uv + 2] - eoff[2 * e_uv];
        const uint64_t s_uw = eoff[2 * e_uw + 2] - eoff[2 * e_uw];
        const uint32_t s_vw = eoff[2 * e_vw + 2] - eoff[2 * e_vw];
        const int k = tri_class(s_uv, s_uw, s_vw, R);
        cls[i] = (uint8_t)k;
#pragma unroll
        for (int x = 0; x < kClasses; ++x) c[x] += k == x;
        acc += (unsigned __int128)(s_uv * s_uw) * s_vw;
        uint64_t b;
        if (k == kClsUnit) {
            b = sizeof(uint4);
        } else {
            const uint32_t probe = 2 * ceil_log2_1(s_vw);
            b = 12 + 36 + 8 * (s_uv + s_uw) + 8 * (uint64_t)(s_vw < probe ? s_vw : probe);
        }
        bytes += b;
        bytes_light += k == kClsLight ? b : 0;
        bytes_medium += (k == kClsMedium || k == kClsContest) ? b : 0;
        bytes_unit += k == kClsUnit ? b : 0;
    }
#pragma unroll
    for (int x = 0; x < kClasses; ++x)
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
    if (threadIdx.x < kClasses) bcnt[kClasses * blockIdx.x + threadIdx.x] = s_cnt[threadIdx.x];
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
// and the totals: tot[0..4] class sizes, tot[5..6] the 128-bit sum of sigma products, tot[7..10]
// the byte totals.
__global__ void __launch_bounds__(kBlock)
k_cls_totals(unsigned nblk, const uint32_t *__restrict__ bcnt, const uint64_t *__restrict__ part,
             uint64_t *__restrict__ base, uint64_t *__restrict__ tot) {
    __shared__ unsigned long long s_tot[kBlock];
    const unsigned tid = threadIdx.x;
    const unsigned per = (nblk + kBlock - 1) / kBlock;
    const unsigned b0 = min(tid * per, nblk), b1 = min(b0 + per, nblk);
    for (int c = 0; c < kClasses; ++c) {
        unsigned long long mine = 0;
        for (unsigned b = b0; b < b1; ++b) mine += bcnt[kClasses * b + c];
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
            base[kClasses * b + c] = run;
            run += bcnt[kClasses * b + c];
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
        tot[kClasses] = (uint64_t)tt;
        tot[kClasses + 1] = (uint64_t)(tt >> 64);
        for (int x = 2; x < kPartWords; ++x) tot[kClasses + x] = tw[x];
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

// Per DAG edge with one temporal edge: that edge's key, with its direction (1: head -> tail) in
// bit 63, which is free while unit records are built (spans below 2^31 and fewer than 2^31 edges
// keep keys below 2^62); all ones for other edges.  The partition then builds a unit record from
// three independent loads instead of three offset-then-key chains.
__global__ void k_unit_keys(uint64_t ms, const uint32_t *__restrict__ eoff, const uint64_t *__restrict__ key,
                            uint64_t *__restrict__ ukey) {
    const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= ms) return;
    const uint32_t a = eoff[2 * e], b = eoff[2 * e + 1], c = eoff[2 * e + 2];
    ukey[e] = c - a == 1 ? key[a] | (uint64_t)(a == b ? 1u : 0u) << 63 : ~0ull;
}

// Every triangle to its class's list at base[class][block] + its rank in the block's walk: unit
// triangles become records (in triangle order) with their t1 bucket as a sort key; light and
// always-medium triangles also go, with their window cell as a sort key, to the windowed copies'
// inputs; always-heavy ones go after the n_c contested ones in the heavy list; contested ones to
// crec for the level search.
__global__ void __launch_bounds__(kBlock)
k_partition(uint64_t n_tri, const uint32_t *__restrict__ tri, const uint8_t *__restrict__ cls,
            const uint64_t *__restrict__ base, const uint32_t *__restrict__ eoff,
            const uint64_t *__restrict__ key, const uint64_t *__restrict__ ukey, int shift, int bshift,
            int cshift, uint64_t n_c,
            uint32_t *__restrict__ light, uint32_t *__restrict__ medium, uint32_t *__restrict__ heavy,
            uint4 *__restrict__ crec, uint4 *__restrict__ lrec, uint16_t *__restrict__ lkey,
            uint4 *__restrict__ mrec, uint16_t *__restrict__ mkey, uint4 *__restrict__ urec,
            uint16_t *__restrict__ ubkt) {
    __shared__ unsigned long long s_wave[kBlock / 64];
    const unsigned lane = threadIdx.x & 63, wave = threadIdx.x / 64;
    uint64_t run[kClasses];
#pragma unroll
    for (int c = 0; c < kClasses; ++c) run[c] = base[kClasses * blockIdx.x + c];
    for (uint64_t b0 = (uint64_t)blockIdx.x * kBlock; b0 < n_tri; b0 += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i = b0 + threadIdx.x;
        const int k = i < n_tri ? cls[i] : kClasses;
        // five 12-bit class counters in one word (a block walks at most 256 triangles per step)
        const unsigned long long f = k < kClasses ? 1ull << (12 * k) : 0ull;
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
        if (k < kClasses) {
            const uint64_t pos = run[k] + (((before + x - f) >> (12 * k)) & 0xfffull);
            const uint32_t e_uv = tri[3 * i], e_uw = tri[3 * i + 1], e_vw = tri[3 * i + 2];
            if (k == kClsUnit) {
                const uint64_t k3[3] = {ukey[e_uv] & ~(1ull << 63), ukey[e_uw] & ~(1ull << 63),
                                        ukey[e_vw] & ~(1ull << 63)};
                const int d3[3] = {(int)(ukey[e_uv] >> 63), (int)(ukey[e_uw] >> 63), (int)(ukey[e_vw] >> 63)};
                const uint4 r = cdev::unit_record_of(k3, d3, shift);
                urec[pos] = r;
                ubkt[pos] = (uint16_t)(r.x >> bshift);
            } else if (k == kClsContest) {
                crec[pos] = make_uint4(e_uv, e_uw, e_vw, 0u);
            } else {
                uint32_t *dst = (k == kClsLight ? light : (k == kClsMedium ? medium : heavy + 3 * n_c)) + 3 * pos;
                dst[0] = e_uv;
                dst[1] = e_uw;
                dst[2] = e_vw;
                if (k == kClsLight) {
                    lrec[pos] = make_uint4(e_uv, e_uw, e_vw, 0u);
                    lkey[pos] = window_cell(e_uv, e_uw, e_vw, eoff, key, shift, cshift);
                } else if (k == kClsMedium) {
                    mrec[pos] = make_uint4(e_uv, e_uw, e_vw, (uint32_t)kLevelAlways);
                    mkey[pos] = window_cell(e_uv, e_uw, e_vw, eoff, key, shift, cshift);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kClasses; ++c) run[c] += (total >> (12 * c)) & 0xfffull;
    }
}

// Level of every contested triangle (one wavefront each): the largest l in 1..kLevels-1 whose
// close pairs -- (x, y) with x on the outer source pair, y on the inner one, |t_x - t_y| <= D(l),
// both directions of both pairs, the whole span -- are at most the triangle's pair budget, or 0.
// The close pairs are counted exactly (two binary searches per outer edge and inner direction) on
// up to kCrossSample outer edges spread evenly over the pair and scaled to all of them, stopping
// once the budget is passed; the levels are found by binary search (close pairs grow with D).
// Writes the level to crec[i].w and the sort key 255 - level (descending levels).  The level only
// decides which exact method counts the triangle for a query.
__global__ void __launch_bounds__(kBlock)
k_crossover(uint64_t nc, uint4 *__restrict__ crec, uint16_t *__restrict__ ckey, const uint32_t *__restrict__ eoff,
            const uint64_t *__restrict__ key, int shift, int64_t span, uint32_t cost_pct) {
    const unsigned lane = threadIdx.x & 63;
    const uint64_t nw = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t i = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / 64; i < nc; i += nw) {
        const uint4 r = crec[i];
        const uint32_t a0 = eoff[2 * r.x], a1 = eoff[2 * r.x + 1], a2 = eoff[2 * r.x + 2];
        const uint32_t b0 = eoff[2 * r.y], b1 = eoff[2 * r.y + 1], b2 = eoff[2 * r.y + 2];
        const uint64_t s_vw = eoff[2 * r.z + 2] - eoff[2 * r.z];
        const double B = pair_budget(a2 - a0, b2 - b0, s_vw, cost_pct);
        const bool outer_uv = cdev::medium_outer_is_uv(a2 - a0, b2 - b0);
        const uint32_t o0 = outer_uv ? a0 : b0, o2 = outer_uv ? a2 : b2;
        const uint32_t i0 = outer_uv ? b0 : a0, i1 = outer_uv ? b1 : a1, i2 = outer_uv ? b2 : a2;
        auto bound = [&](int64_t x) -> uint64_t {   // key bound of "t < x" (relative times)
            return x <= 0 ? 0ull : (x > span ? ~0ull : ((uint64_t)x << shift));
        };
        const uint32_t n_out = o2 - o0;
        const uint32_t n_s = n_out < kCrossSample ? n_out : kCrossSample;
        const double scale = n_s ? (double)n_out / n_s : 0.0;
        // within the budget at distance D (the same answer in every lane)
        auto fits = [&](int64_t D) -> bool {
            unsigned long long c = 0;
            for (uint32_t s0 = 0; s0 < n_s; s0 += 64) {
                const uint32_t si = s0 + lane;
                if (si < n_s) {
                    const uint32_t x = o0 + (uint32_t)(((uint64_t)si * n_out) / n_s);
                    const int64_t tx = (int64_t)(key[x] >> shift);
                    const uint64_t klo = bound(tx - D), khi = bound(tx + D + 1);
                    uint32_t l0, h0, l1, h1;
                    cdev::lower2(key, i0, i1, klo, khi, l0, h0);
                    cdev::lower2(key, i1, i2, klo, khi, l1, h1);
                    c += (h0 - l0) + (h1 - l1);
                }
                if ((double)cdev::wave_sum(c) * scale > B) return false;
            }
            return true;
        };
        uint32_t lo = 0, hi = kLevels - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            if (fits(level_delta(mid))) lo = mid;
            else hi = mid - 1;
        }
        if (lane == 0) {
            crec[i].w = lo;
            ckey[i] = (uint16_t)(255u - lo);
        }
    }
}

// The contested triangles in descending level order (crec sorted): after the n_a always-medium
// ones in the medium list (with their window cells and levels for the windowed copy) and first in
// the heavy list.
__global__ void k_contest_place(uint64_t nc, const uint4 *__restrict__ crec, uint64_t n_a,
                                uint32_t *__restrict__ medium, uint32_t *__restrict__ heavy, uint4 *__restrict__ mrec,
                                uint16_t *__restrict__ mkey, const uint32_t *__restrict__ eoff,
                                const uint64_t *__restrict__ key, int shift, int cshift) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nc) return;
    const uint4 r = crec[i];
    const uint64_t m = n_a + i;
    medium[3 * m] = r.x;
    medium[3 * m + 1] = r.y;
    medium[3 * m + 2] = r.z;
    heavy[3 * i] = r.x;
    heavy[3 * i + 1] = r.y;
    heavy[3 * i + 2] = r.z;
    mrec[m] = r;
    mkey[m] = window_cell(r.x, r.y, r.z, eoff, key, shift, cshift);
}

// bucket starts from the sorted bucket keys: start[x] for every x in (key[j - 1], key[j]] is j;
// j = nu closes the array at nbk
// first position of every bucket 0..nbk in the nu sorted bucket keys (a binary search per bucket;
// nu for nbk and for buckets past the last key)
__global__ void k_unit_starts(uint64_t nu, uint32_t nbk, const uint16_t *__restrict__ bkt,
                              uint32_t *__restrict__ start) {
    const uint32_t x = blockIdx.x * kBlock + threadIdx.x;
    if (x > nbk) return;
    uint64_t lo = 0, len = nu;
    while (len > 0) {
        const uint64_t half = len >> 1;
        if (bkt[lo + half] < x) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    start[x] = (uint32_t)lo;
}

// first position of every key value 0..nk-1 in a sorted key array (nk + 1 entries, the last = n)
__global__ void k_key_starts(uint64_t n, uint32_t nk, const uint16_t *__restrict__ ck, uint64_t *__restrict__ start) {
    uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j > n) return;
    const int64_t cur = j < n ? (int64_t)ck[j] : (int64_t)nk;
    const int64_t prev = j > 0 ? (int64_t)ck[j - 1] : -1;
    for (int64_t x = prev + 1; x <= cur; ++x) start[x] = j;
}

// (e_uv, e_uw, e_vw, level) records back to three words per triangle (and the levels to lev)
__global__ void k_unpack3(uint64_t n, const uint4 *__restrict__ rec, uint32_t *__restrict__ out,
                          uint8_t *__restrict__ lev) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint4 r = rec[i];
    out[3 * i] = r.x;
    out[3 * i + 1] = r.y;
    out[3 * i + 2] = r.z;
    if (lev) lev[i] = (uint8_t)r.w;
}

// first medium item of every cell: the item base of the cell's first triangle
__global__ void k_cell_items(const uint64_t *__restrict__ tstart, const uint64_t *__restrict__ ibase,
                             uint64_t *__restrict__ istart) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c <= kCells) istart[c] = ibase[tstart[c]];
}

// entries of the medium path: one per edge of the outer pair (the source-incident pair with fewer
// temporal edges) and chunk of the inner pair
__global__ void k_medium_sizes(uint64_t nm, const uint32_t *__restrict__ med, const uint32_t *__restrict__ eoff,
                               uint64_t *__restrict__ nch) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nm) return;
    const uint32_t e_uv = med[3 * i], e_uw = med[3 * i + 1];
    const uint32_t s_uv = eoff[2 * e_uv + 2] - eoff[2 * e_uv], s_uw = eoff[2 * e_uw + 2] - eoff[2 * e_uw];
    const bool outer_uv = cdev::medium_outer_is_uv(s_uv, s_uw);
    const uint32_t s_out = outer_uv ? s_uv : s_uw, s_in = outer_uv ? s_uw : s_uv;
    nch[i] = (uint64_t)s_out * cdev::medium_inner_chunks(s_out, s_in);
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

constexpr uint32_t kChunk = 256;   // source edges per count chunk and per prefix chunk

// prefix slots (four arrays of length sigma + 1), count chunks and prefix chunks (at least one per
// list, so that an empty list's total is written too) of every heavy triangle
__global__ void k_heavy_sizes(uint64_t n_heavy, const uint32_t *__restrict__ heavy,
                              const uint32_t *__restrict__ eoff, uint64_t *__restrict__ slots,
                              uint64_t *__restrict__ nch, uint64_t *__restrict__ npch) {
    uint64_t h = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (h >= n_heavy) return;
    const uint32_t e_uv = heavy[3 * h], e_uw = heavy[3 * h + 1];
    const uint32_t len[4] = {eoff[2 * e_uv + 1] - eoff[2 * e_uv], eoff[2 * e_uv + 2] - eoff[2 * e_uv + 1],
                             eoff[2 * e_uw + 1] - eoff[2 * e_uw], eoff[2 * e_uw + 2] - eoff[2 * e_uw + 1]};
    const uint64_t src = (uint64_t)len[0] + len[1] + len[2] + len[3];
    slots[h] = src + 4;
    nch[h] = (src + kChunk - 1) / kChunk;
    uint64_t p = 0;
    for (int X = 0; X < 4; ++X) p += len[X] ? (len[X] + kChunk - 1) / kChunk : 1;
    npch[h] = p;
}

__global__ void k_heavy_chunks(uint64_t n_heavy, const uint32_t *__restrict__ heavy, const uint32_t *__restrict__ eoff,
                               const uint64_t *__restrict__ nch, const uint64_t *__restrict__ cbase,
                               const uint64_t *__restrict__ pbase, uint32_t *__restrict__ chunks,
                               uint32_t *__restrict__ pchunks) {
    uint64_t h = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (h >= n_heavy) return;
    for (uint64_t j = 0; j < nch[h]; ++j) {
        chunks[2 * (cbase[h] + j)] = (uint32_t)h;
        chunks[2 * (cbase[h] + j) + 1] = (uint32_t)(j * kChunk);
    }
    const uint32_t e_uv = heavy[3 * h], e_uw = heavy[3 * h + 1];
    const uint32_t len[4] = {eoff[2 * e_uv + 1] - eoff[2 * e_uv], eoff[2 * e_uv + 2] - eoff[2 * e_uv + 1],
                             eoff[2 * e_uw + 1] - eoff[2 * e_uw], eoff[2 * e_uw + 2] - eoff[2 * e_uw + 1]};
    uint64_t p = pbase[h];
    for (uint32_t X = 0; X < 4; ++X) {
        const uint32_t nc = len[X] ? (len[X] + kChunk - 1) / kChunk : 1;
        for (uint32_t c = 0; c < nc; ++c, ++p) {
            pchunks[2 * p] = (uint32_t)h;
            pchunks[2 * p + 1] = c * kChunk | X;
        }
    }
}

// Per query level l = 1..kLevels, from the contested triangles' level starts (kstart over the
// descending sort keys 255 - level): c = contested triangles of level >= l; the medium entries end
// at ibase[n_a + c]; the heavy triangles, count chunks, prefix chunks and slots start at c.
__global__ void k_level_tables(uint64_t n_a, const uint64_t *__restrict__ kstart, const uint64_t *__restrict__ ibase,
                               const uint64_t *__restrict__ cbase, const uint64_t *__restrict__ pbase,
                               const uint64_t *__restrict__ hslot, uint64_t *__restrict__ out) {
    const uint32_t l = threadIdx.x;
    if (l == 0 || l > kLevels) return;
    const uint64_t c = kstart[256 - l];
    out[0 * (kLevels + 1) + l] = ibase[n_a + c];
    out[1 * (kLevels + 1) + l] = c;
    out[2 * (kLevels + 1) + l] = cbase[c];
    out[3 * (kLevels + 1) + l] = pbase[c];
    out[4 * (kLevels + 1) + l] = hslot[c];
}

// Sort n (cell, record) pairs by cell, unpack the records to out (three words per triangle) and
// write the cell starts (kCells + 1 entries) to start
// (and, with lev, the records' levels to lev)
int cell_order(dt_ctx *ctx, uint64_t n, DevMem &ckey, DevMem &rec, DevMem &out, DevMem &start, hipStream_t st,
               uint8_t *lev = nullptr) {
    DevMem k2, r2;
    DT_TRY(dev_alloc(ctx, start, (uint64_t)(kCells + 1) * 8));
    DT_TRY(dev_alloc(ctx, k2, n * 2));
    DT_TRY(dev_alloc(ctx, r2, n * sizeof(uint4)));
    DT_TRY(sort_pairs_u16_u4(ctx, ckey.as<uint16_t>(), k2.as<uint16_t>(), rec.as<uint4>(), r2.as<uint4>(), n, 16, st));
    k_key_starts<<<grid_for(n + 1, kBlock), kBlock, 0, st>>>(n, kCells, k2.as<uint16_t>(), start.as<uint64_t>());
    DT_HIP(hipGetLastError());
    if (n) {
        k_unpack3<<<grid_for(n, kBlock), kBlock, 0, st>>>(n, r2.as<uint4>(), out.as<uint32_t>(), lev);
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
    const uint64_t nt = g->n_tri_list;   // list entries (empty ones have no class)
    Schedule &S = g->sched;
    S = Schedule();
    SplitRule R;
    R.cap_l = g->light_cap_used ? g->light_cap_used : 4;
    R.cap_m = g->tuning.medium_pair_cap;
    R.force = g->tuning.force_path;
    R.cost_pct = g->cost_pct_used ? g->cost_pct_used : 100;
    // unit records hold 32-bit relative times
    R.unit_ok = g->span <= kUnitMaxSpan ? 1u : 0u;
    const unsigned grid = kClsGrid;
    DevMem cls, bcnt, part, base;
    DT_TRY(dev_alloc(ctx, cls, nt + 1));
    DT_TRY(dev_alloc(ctx, bcnt, (uint64_t)grid * kClasses * 4));
    DT_TRY(dev_alloc(ctx, part, (uint64_t)grid * kPartWords * 8));
    DT_TRY(dev_alloc(ctx, base, (uint64_t)grid * kClasses * 8));
    // the per-edge unit keys (when unit records are allowed) on the first side stream, beside the
    // classify pass; the partition pass waits for them
    const bool units = R.force == 0 && R.unit_ok && g->m_s;
    const hipStream_t ks = units && ctx->side[0] ? ctx->side[0] : st;
    DevMem ukey;
    DT_TRY(dev_alloc(ctx, ukey, (units ? g->m_s : 0) * 8));
    struct KeyJoin {   // an early return must not release ukey while the side stream writes it
        hipStream_t s, main;
        ~KeyJoin() {
            if (s != main) (void)hipStreamSynchronize(s);
        }
    } kjoin{ks, st};
    if (units) {
        if (ks != st) {
            DT_HIP(hipEventRecord(ctx->ev_relay[0], st));
            DT_HIP(hipStreamWaitEvent(ks, ctx->ev_relay[0], 0));
        }
        k_unit_keys<<<grid_for(g->m_s, kBlock), kBlock, 0, ks>>>(g->m_s, g->eoff.as<uint32_t>(), g->key.as<uint64_t>(),
                                                                 ukey.as<uint64_t>());
        DT_HIP(hipGetLastError());
        if (ks != st) DT_HIP(hipEventRecord(ctx->ev_relay[1], ks));
    }
    k_classify<<<grid, kBlock, 0, st>>>(nt, tri.as<uint32_t>(), g->eoff.as<uint32_t>(), R, cls.as<uint8_t>(),
                                        bcnt.as<uint32_t>(), part.as<uint64_t>());
    DT_HIP(hipGetLastError());
    DevMem tot;
    DT_TRY(dev_alloc(ctx, tot, 16 * 8));
    k_cls_totals<<<1, kBlock, 0, st>>>(grid, bcnt.as<uint32_t>(), part.as<uint64_t>(), base.as<uint64_t>(),
                                       tot.as<uint64_t>());
    DT_HIP(hipGetLastError());
    uint64_t *hs = reinterpret_cast<uint64_t *>(ctx->pinned_stage);
    DT_HIP(hipMemcpyAsync(hs, tot.ptr, kTotWords * 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    uint64_t ncls[kClasses];
    for (int c = 0; c < kClasses; ++c) ncls[c] = hs[c];
    const unsigned __int128 s3 = ((unsigned __int128)hs[kClasses + 1] << 64) | hs[kClasses];
    g->sum_sigma3 = s3;
    g->alg_bytes = hs[kClasses + 2];
    g->alg_bytes_light = hs[kClasses + 3];
    g->alg_bytes_medium = hs[kClasses + 4];
    g->alg_bytes_unit = hs[kClasses + 5];
    const uint64_t na = ncls[kClsMedium], nh_always = ncls[kClsHeavy], nu = ncls[kClsUnit], nc = ncls[kClsContest];
    if (ncls[kClsLight] + na + nh_always + nu + nc != g->n_tri)
        return fail(DT_EDEVICE, "triangle classes do not add up");
    S.n_light = ncls[kClsLight];
    S.n_always_medium = na;
    S.n_contested = nc;
    S.n_always_heavy = nh_always;
    S.n_medium = na + nc;
    S.n_heavy = nc + nh_always;
    S.n_unit = nu;
    const uint64_t nm = S.n_medium, nh = S.n_heavy;
    DT_TRY(dev_alloc(ctx, S.light, S.n_light * 12));
    DT_TRY(dev_alloc(ctx, S.medium, nm * 12));
    DT_TRY(dev_alloc(ctx, S.heavy, nh * 12));
    // t1 buckets of the unit records: at most 2^16, t1 >> unit_shift
    int t_bits = 0;
    while (t_bits < 31 && (1ll << t_bits) <= g->span) ++t_bits;
    S.unit_shift = t_bits > 16 ? t_bits - 16 : 0;
    const uint64_t nbk = R.unit_ok ? ((uint64_t)g->span >> S.unit_shift) + 1 : 1;
    // time slices of the window index: span >> cell_shift < kSlices
    S.cell_shift = 0;
    while (S.cell_shift < 62 && (g->span >> S.cell_shift) >= (int64_t)kSlices) ++S.cell_shift;
    DevMem urec, ubkt, ubkt2, ustart, lrec, lkey, mrec, mkey, lstart, mstart, crec, ckey;
    DT_TRY(dev_alloc(ctx, urec, nu * sizeof(uint4)));
    DT_TRY(dev_alloc(ctx, ubkt, nu * 2));
    DT_TRY(dev_alloc(ctx, lrec, S.n_light * sizeof(uint4)));
    DT_TRY(dev_alloc(ctx, lkey, S.n_light * 2));
    DT_TRY(dev_alloc(ctx, mrec, nm * sizeof(uint4)));
    DT_TRY(dev_alloc(ctx, mkey, nm * 2));
    DT_TRY(dev_alloc(ctx, crec, nc * sizeof(uint4)));
    DT_TRY(dev_alloc(ctx, ckey, nc * 2));
    if (units && ks != st) DT_HIP(hipStreamWaitEvent(st, ctx->ev_relay[1], 0));
    if (nt) {
        k_partition<<<grid, kBlock, 0, st>>>(nt, tri.as<uint32_t>(), cls.as<uint8_t>(), base.as<uint64_t>(),
            g->eoff.as<uint32_t>(), g->key.as<uint64_t>(), ukey.as<uint64_t>(), g->shift, S.unit_shift, S.cell_shift, nc,
            S.light.as<uint32_t>(), S.medium.as<uint32_t>(), S.heavy.as<uint32_t>(), crec.as<uint4>(), lrec.as<uint4>(),
            lkey.as<uint16_t>(), mrec.as<uint4>(), mkey.as<uint16_t>(), urec.as<uint4>(), ubkt.as<uint16_t>());
        DT_HIP(hipGetLastError());
    }
    cls.reset();
    ukey.reset();
    // unit records ordered by t1 bucket (a stable two-pass radix sort on the 16-bit bucket) on the
    // first side stream, while this stream builds the other lists; the host keeps the bucket starts
    // (read back through the pinned staging buffer from byte kStageUnit; the cell starts, level
    // tables and other read-backs use the bytes before it)
    constexpr size_t kStageUnit = 16384;
    static_assert((kCells + 1) * 8 <= kStageUnit, "staging layout");
    static_assert(5 * (kLevels + 1) * 8 + 16 <= kStageUnit, "staging layout");
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
        k_unit_starts<<<grid_for(nbk + 1, kBlock), kBlock, 0, us>>>(nu, (uint32_t)nbk, ubkt2.as<uint16_t>(),
                                                                    ustart.as<uint32_t>());
        DT_HIP(hipGetLastError());
        S.unit_index.resize(nbk + 1);
        DT_HIP(hipMemcpyAsync(ctx->pinned_stage + kStageUnit, ustart.ptr, (nbk + 1) * 4, hipMemcpyDeviceToHost, us));
        if (us != st) DT_HIP(hipEventRecord(ctx->ev_relay[1], us));
    }
    // contested triangles: their levels, then descending level order after the always-medium
    // ones (medium list) and before the always-heavy ones (heavy list)
    DevMem kstart;
    DT_TRY(dev_alloc(ctx, kstart, 257 * 8));
    {
        DevMem ckey2, crec2;
        DT_TRY(dev_alloc(ctx, ckey2, nc * 2));
        DT_TRY(dev_alloc(ctx, crec2, nc * sizeof(uint4)));
        if (nc) {
            k_crossover<<<(unsigned)std::min<uint64_t>((nc + kBlock / 64 - 1) / (kBlock / 64), (uint64_t)ctx->num_cus * 16),
                          kBlock, 0, st>>>(nc, crec.as<uint4>(), ckey.as<uint16_t>(), g->eoff.as<uint32_t>(),
                                           g->key.as<uint64_t>(), g->shift, g->span, R.cost_pct);
            DT_HIP(hipGetLastError());
            DT_TRY(sort_pairs_u16_u4(ctx, ckey.as<uint16_t>(), ckey2.as<uint16_t>(), crec.as<uint4>(), crec2.as<uint4>(),
                                     nc, 16, st));
            k_contest_place<<<grid_for(nc, kBlock), kBlock, 0, st>>>(nc, crec2.as<uint4>(), na, S.medium.as<uint32_t>(),
                S.heavy.as<uint32_t>(), mrec.as<uint4>(), mkey.as<uint16_t>(), g->eoff.as<uint32_t>(),
                g->key.as<uint64_t>(), g->shift, S.cell_shift);
            DT_HIP(hipGetLastError());
        }
        k_key_starts<<<grid_for(nc + 1, kBlock), kBlock, 0, st>>>(nc, 256, ckey2.as<uint16_t>(), kstart.as<uint64_t>());
        DT_HIP(hipGetLastError());
    }
    crec.reset();
    ckey.reset();
    // the windowed copies of the light and medium lists, in window-cell order
    DT_TRY(dev_alloc(ctx, S.light_w, S.n_light * 12));
    DT_TRY(dev_alloc(ctx, S.medium_w, nm * 12));
    DT_TRY(dev_alloc(ctx, S.mlev_w, nm + 1));
    DT_TRY(cell_order(ctx, S.n_light, lkey, lrec, S.light_w, lstart, st));
    DT_TRY(cell_order(ctx, nm, mkey, mrec, S.medium_w, mstart, st, S.mlev_w.as<uint8_t>()));
    S.light_cells.resize(kCells + 1);
    DT_HIP(hipMemcpyAsync(ctx->pinned_stage, lstart.ptr, (kCells + 1) * 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    memcpy(S.light_cells.data(), ctx->pinned_stage, (kCells + 1) * 8);
    // medium work items of both copies (the same totals: the same triangles in another order)
    DevMem nch0, base0;
    {
        DevMem nch1, base;
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
    // heavy slots, count chunks and prefix chunks
    DevMem slots, nch, npch, cbase, pbase;
    DT_TRY(dev_alloc(ctx, slots, (nh + 1) * 8));
    DT_TRY(dev_alloc(ctx, nch, (nh + 1) * 8));
    DT_TRY(dev_alloc(ctx, npch, (nh + 1) * 8));
    DT_TRY(dev_alloc(ctx, cbase, (nh + 1) * 8));
    DT_TRY(dev_alloc(ctx, pbase, (nh + 1) * 8));
    DT_TRY(dev_alloc(ctx, S.hslot, (nh + 1) * 8));
    DT_HIP(hipMemsetAsync(slots.ptr, 0, (nh + 1) * 8, st));
    DT_HIP(hipMemsetAsync(nch.ptr, 0, (nh + 1) * 8, st));
    DT_HIP(hipMemsetAsync(npch.ptr, 0, (nh + 1) * 8, st));
    if (nh) {
        k_heavy_sizes<<<grid_for(nh, kBlock), kBlock, 0, st>>>(nh, S.heavy.as<uint32_t>(), g->eoff.as<uint32_t>(),
                                                               slots.as<uint64_t>(), nch.as<uint64_t>(), npch.as<uint64_t>());
        DT_HIP(hipGetLastError());
    }
    DT_TRY(exclusive_scan_u64(ctx, slots.as<uint64_t>(), S.hslot.as<uint64_t>(), nh + 1, st));
    DT_TRY(exclusive_scan_u64(ctx, nch.as<uint64_t>(), cbase.as<uint64_t>(), nh + 1, st));
    DT_TRY(exclusive_scan_u64(ctx, npch.as<uint64_t>(), pbase.as<uint64_t>(), nh + 1, st));
    uint64_t *htot = reinterpret_cast<uint64_t *>(ctx->pinned_stage);
    DT_HIP(hipMemcpyAsync(&htot[0], S.hslot.as<uint64_t>() + nh, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipMemcpyAsync(&htot[1], cbase.as<uint64_t>() + nh, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipMemcpyAsync(&htot[2], pbase.as<uint64_t>() + nh, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    S.n_slots = htot[0];
    S.n_chunks = htot[1];
    S.n_pchunks = htot[2];
    if (S.n_chunks > 0xffffffffull || S.n_pchunks > 0xffffffffull || nh > 0xffffffffull)
        return fail(DT_EOVERFLOW, "too many heavy work items (%llu)", (unsigned long long)S.n_chunks);
    DT_TRY(dev_alloc(ctx, S.chunks, S.n_chunks * 8));
    DT_TRY(dev_alloc(ctx, S.pchunks, S.n_pchunks * 8));
    if (nh) {
        k_heavy_chunks<<<grid_for(nh, kBlock), kBlock, 0, st>>>(nh, S.heavy.as<uint32_t>(), g->eoff.as<uint32_t>(),
                                                                nch.as<uint64_t>(), cbase.as<uint64_t>(),
                                                                pbase.as<uint64_t>(), S.chunks.as<uint32_t>(),
                                                                S.pchunks.as<uint32_t>());
        DT_HIP(hipGetLastError());
    }
    // the per-level bounds of the two lists
    {
        DevMem lt;
        DT_TRY(dev_alloc(ctx, lt, 5 * (kLevels + 1) * 8));
        DT_HIP(hipMemsetAsync(lt.ptr, 0, 5 * (kLevels + 1) * 8, st));
        k_level_tables<<<1, 64, 0, st>>>(na, kstart.as<uint64_t>(), base0.as<uint64_t>(), cbase.as<uint64_t>(),
                                         pbase.as<uint64_t>(), S.hslot.as<uint64_t>(), lt.as<uint64_t>());
        DT_HIP(hipGetLastError());
        DT_HIP(hipMemcpyAsync(htot, lt.ptr, 5 * (kLevels + 1) * 8, hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
        for (uint32_t l = 1; l <= kLevels; ++l) {
            S.med_item_at[l] = htot[0 * (kLevels + 1) + l];
            S.heavy_tri_at[l] = htot[1 * (kLevels + 1) + l];
            S.heavy_chunk_at[l] = htot[2 * (kLevels + 1) + l];
            S.heavy_pchunk_at[l] = htot[3 * (kLevels + 1) + l];
            S.heavy_slot_at[l] = htot[4 * (kLevels + 1) + l];
        }
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
