// Device-side building blocks of the count, shared by the single-query kernels (count.hip) and the
// batched kernel (batch.hip).  See count.hip for the method.
#pragma once

#include "internal.h"

namespace dt {
namespace cdev {

// ---------------------------------------------------------------------------------------------
// cell and type tables
// ---------------------------------------------------------------------------------------------
// Figure 4: orientation number from the direction bit of each pair (0 = from the earlier vertex
// of the ordering u < v < w, 1 = towards it).
__host__ __device__ constexpr int rho_of(int d_uv, int d_uw, int d_vw) {
    constexpr int tab[8] = {/*000*/ 1, /*001*/ 3, /*010*/ 4, /*011*/ 2,
                            /*100*/ 5, /*101*/ 7, /*110*/ 8, /*111*/ 6};
    return tab[(d_uv << 2) | (d_uw << 1) | d_vw];
}

// Table 2: psi[pi - 1][rho - 1] = type.
__host__ __device__ constexpr int psi_of(int pi, int rho) {
    constexpr int tab[6][8] = {
        {7, 6, 5, 8, 3, 2, 4, 1},
        {5, 3, 7, 4, 6, 1, 8, 2},
        {3, 2, 1, 4, 7, 6, 8, 5},
        {1, 7, 3, 8, 2, 5, 4, 6},
        {6, 1, 2, 8, 5, 3, 4, 7},
        {2, 5, 6, 4, 1, 7, 8, 3},
    };
    return tab[pi - 1][rho - 1];
}

// 0-based type index and cell index of (pi, direction bits)
template <int PI, int DUV, int DUW, int DVW> struct Cell {
    static constexpr int rho = rho_of(DUV, DUW, DVW);
    static constexpr int type = psi_of(PI, rho) - 1;
    static constexpr int cell = (PI - 1) * 8 + (rho - 1);
};

// accumulators: per-lane type counts, or (diagnostic) global atomics per cell
template <bool CELLS> struct Acc;
// `visits` counts the (uv edge, uw edge) pairs or list elements a lane iterated over (the work
// measure of Theorem 1's bound; reported by the instrumented count).
template <> struct Acc<false> {
    int64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t *cells = nullptr;
    uint64_t visits = 0;
    template <class CA, class CB> __device__ __forceinline__ void add2(bool first, int64_t v) {
        t[CA::type] += first ? v : 0;
        t[CB::type] += first ? 0 : v;
    }
    template <class C> __device__ __forceinline__ void add(int64_t v) { t[C::type] += v; }
};
template <> struct Acc<true> {
    int64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t *cells = nullptr;
    uint64_t visits = 0;
    template <class CA, class CB> __device__ __forceinline__ void add2(bool first, int64_t v) {
        if (v) atomicAdd((unsigned long long *)(cells + (first ? CA::cell : CB::cell)),
                         (unsigned long long)v);
    }
    template <class C> __device__ __forceinline__ void add(int64_t v) {
        if (v) atomicAdd((unsigned long long *)(cells + C::cell), (unsigned long long)v);
    }
};

// 128-bit per-lane type counts, for graphs whose sum of multiplicity products reaches 2^63 (every
// contribution is non-negative, so the sums only need more bits, never a sign)
struct AccW {
    unsigned __int128 t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t *cells = nullptr;
    uint64_t visits = 0;
    template <class CA, class CB> __device__ __forceinline__ void add2(bool first, int64_t v) {
        t[CA::type] += first ? (unsigned __int128)(uint64_t)v : 0;
        t[CB::type] += first ? 0 : (unsigned __int128)(uint64_t)v;
    }
    template <class C> __device__ __forceinline__ void add(int64_t v) { t[C::type] += (uint64_t)v; }
};

// position of element j of the ranges R (j < R.pre[R.n]); the cursor r only moves forward, so a
// thread walking increasing j finds each range once
__device__ __forceinline__ uint64_t range_at(const Ranges &R, uint32_t &r, uint64_t j) {
    while (j >= R.pre[r + 1]) ++r;
    return R.b[r] + (j - R.pre[r]);
}

// ---------------------------------------------------------------------------------------------
// searches on key-sorted lists
// ---------------------------------------------------------------------------------------------
// first index in [lo, hi) whose key is >= K (hi if none); the bounds 0 and ~0 (times before or
// after the whole span, common at long deltas) need no search
__device__ __forceinline__ uint32_t lower(const uint64_t *__restrict__ key, uint32_t lo, uint32_t hi,
                                          uint64_t K) {
    if (K == 0) return lo;
    if (K == ~0ull) return hi;
    uint32_t len = hi - lo;
    while (len > 0) {
        uint32_t half = len >> 1;
        if (key[lo + half] < K) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

// key bound of "t < x" for a relative time x
__device__ __forceinline__ uint64_t before_time(int64_t x, const DQuery &q) {
    return x <= 0 ? 0ull : (x > q.span ? ~0ull : ((uint64_t)x << q.shift));
}

struct Lists {
    uint32_t lo[6], hi[6];   // uv+, uv-, uw+, uw-, vw+, vw- (clipped to the window)
};

__device__ __forceinline__ void load_lists(const uint32_t *__restrict__ eoff, uint32_t e_uv,
                                           uint32_t e_uw, uint32_t e_vw, const uint64_t *__restrict__ key,
                                           const DQuery &q, Lists &L) {
    const uint32_t es[3] = {e_uv, e_uw, e_vw};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        uint32_t a = eoff[2 * es[p]], b = eoff[2 * es[p] + 1], c = eoff[2 * es[p] + 2];
        L.lo[2 * p] = a;
        L.hi[2 * p] = b;
        L.lo[2 * p + 1] = b;
        L.hi[2 * p + 1] = c;
    }
    if (q.windowed) {
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            uint32_t lo = L.lo[i], hi = L.hi[i];
            L.lo[i] = lower(key, lo, hi, q.klo);
            L.hi[i] = lower(key, L.lo[i], hi, q.khi);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// light path: one lane per triangle, every (uv edge, uw edge) pair
// ---------------------------------------------------------------------------------------------
template <int A, int B, int C, class ACC>
__device__ __forceinline__ void light_third(const uint64_t *__restrict__ key, const Lists &L,
                                            const DQuery &q, bool uv_first, uint64_t k_lo,
                                            uint64_t k_hi, int64_t t_lo, int64_t t_hi, int64_t gap,
                                            ACC &acc) {
    const uint32_t zb = L.lo[4 + C], ze = L.hi[4 + C];
    if (zb == ze) return;
    const uint32_t below_lo = lower(key, zb, ze, k_lo);   // z with key < k_lo
    const uint32_t below_hi = lower(key, below_lo, ze, k_hi);
    // z first: e1 = z, e2 = earlier of x, y, e3 = later
    if (gap <= q.d23) {
        int64_t from = t_lo - q.d12 > t_hi - q.d13 ? t_lo - q.d12 : t_hi - q.d13;
        uint32_t s = lower(key, zb, below_lo, before_time(from, q));
        acc.template add2<Cell<5, A, B, C>, Cell<6, A, B, C>>(uv_first, (int64_t)(below_lo - s));
    }
    // z in the middle: t_hi - d23 <= t_z <= t_lo + d12, key between k_lo and k_hi
    {
        uint32_t a = lower(key, below_lo, below_hi, before_time(t_hi - q.d23, q));
        uint32_t b = lower(key, below_lo, below_hi, before_time(t_lo + q.d12 + 1, q));
        if (b > a) acc.template add2<Cell<3, A, B, C>, Cell<4, A, B, C>>(uv_first, (int64_t)(b - a));
    }
    // z last: t_z <= min(t_hi + d23, t_lo + d13), key after k_hi
    if (gap <= q.d12) {
        int64_t until = t_hi + q.d23 < t_lo + q.d13 ? t_hi + q.d23 : t_lo + q.d13;
        uint32_t e = lower(key, below_hi, ze, before_time(until + 1, q));
        acc.template add2<Cell<1, A, B, C>, Cell<2, A, B, C>>(uv_first, (int64_t)(e - below_hi));
    }
}

template <int A, int B, class ACC>
__device__ __forceinline__ void light_pairs(const uint64_t *__restrict__ key, const Lists &L,
                                            const DQuery &q, ACC &acc) {
    const uint32_t xb = L.lo[A], xe = L.hi[A], yb = L.lo[2 + B], ye = L.hi[2 + B];
    acc.visits += (uint64_t)(xe - xb) * (ye - yb);
    for (uint32_t ix = xb; ix < xe; ++ix) {
        const uint64_t kx = key[ix];
        for (uint32_t iy = yb; iy < ye; ++iy) {
            const uint64_t ky = key[iy];
            const bool uv_first = kx < ky;
            const uint64_t k_lo = uv_first ? kx : ky, k_hi = uv_first ? ky : kx;
            const int64_t t_lo = (int64_t)(k_lo >> q.shift), t_hi = (int64_t)(k_hi >> q.shift);
            const int64_t gap = t_hi - t_lo;
            if (gap > q.d13) continue;   // d12, d23 <= d13: no z completes this pair
            light_third<A, B, 0>(key, L, q, uv_first, k_lo, k_hi, t_lo, t_hi, gap, acc);
            light_third<A, B, 1>(key, L, q, uv_first, k_lo, k_hi, t_lo, t_hi, gap, acc);
        }
    }
}

// one light triangle: every (uv edge, uw edge) pair by one lane
template <class ACC>
__device__ __forceinline__ void light_tri(const uint32_t *__restrict__ tri, uint64_t i,
                                          const uint32_t *__restrict__ eoff,
                                          const uint64_t *__restrict__ key, const DQuery &q,
                                          ACC &acc) {
    Lists L;
    load_lists(eoff, tri[3 * i], tri[3 * i + 1], tri[3 * i + 2], key, q, L);
    light_pairs<0, 0>(key, L, q, acc);
    light_pairs<0, 1>(key, L, q, acc);
    light_pairs<1, 0>(key, L, q, acc);
    light_pairs<1, 1>(key, L, q, acc);
}

// ---------------------------------------------------------------------------------------------
// medium path: one lane per edge of a triangle's smaller source-incident pair
// ---------------------------------------------------------------------------------------------
template <int A, int B, class ACC>
__device__ __forceinline__ void medium_pair(const uint64_t *__restrict__ key, const Lists &L,
                                            const DQuery &q, uint64_t kx, uint64_t ky, ACC &acc) {
    const bool uv_first = kx < ky;
    const uint64_t k_lo = uv_first ? kx : ky, k_hi = uv_first ? ky : kx;
    const int64_t t_lo = (int64_t)(k_lo >> q.shift), t_hi = (int64_t)(k_hi >> q.shift);
    const int64_t gap = t_hi - t_lo;
    if (gap > q.d13) return;
    light_third<A, B, 0>(key, L, q, uv_first, k_lo, k_hi, t_lo, t_hi, gap, acc);
    light_third<A, B, 1>(key, L, q, uv_first, k_lo, k_hi, t_lo, t_hi, gap, acc);
}

// the outer pair of a medium triangle: the source-incident pair with fewer temporal edges
// (uv on a tie); the medium path has one entry per outer edge
__host__ __device__ __forceinline__ bool medium_outer_is_uv(uint32_t s_uv, uint32_t s_uw) { return s_uv <= s_uw; }

// A medium entry is one outer edge and, when the inner pair is long, one chunk of kInnerChunk of
// the inner pair's edges (indices over its direction-0 run followed by its direction-1 run): no
// entry then has more than kInnerChunk close pairs at any delta, and the wavefronts that take the
// consecutive entries of a triangle with a short and a long source pair share its pairs instead of
// one of them walking all of them.  Only triangles with at most kChunkMaxPairs pairs are split
// (each chunk is an entry, searched at every delta); the triangle's entries are its outer edges
// times its chunks, entry j' standing for outer edge j' / chunks and chunk j' % chunks.
constexpr uint32_t kInnerChunk = 512;
constexpr uint64_t kChunkMaxPairs = 1ull << 20;
__host__ __device__ __forceinline__ uint32_t medium_inner_chunks(uint32_t s_outer, uint32_t s_inner) {
    return s_inner > kInnerChunk && (uint64_t)s_outer * s_inner <= kChunkMaxPairs
               ? (s_inner + kInnerChunk - 1) / kInnerChunk
               : 1u;
}

// first indices in [lo, hi) whose keys are >= K1 and >= K2 (two searches in one loop)
__device__ __forceinline__ void lower2(const uint64_t *__restrict__ key, uint32_t lo, uint32_t hi, uint64_t K1,
                                       uint64_t K2, uint32_t &r1, uint32_t &r2) {
    uint32_t l1 = lo, l2 = lo, len1 = hi - lo, len2 = hi - lo;
    while (len1 | len2) {
        const uint32_t h1 = len1 >> 1, h2 = len2 >> 1;
        const bool go1 = len1 && key[l1 + h1] < K1, go2 = len2 && key[l2 + h2] < K2;
        l1 += go1 ? h1 + 1 : 0;
        len1 = go1 ? len1 - h1 - 1 : h1;
        l2 += go2 ? h2 + 1 : 0;
        len2 = go2 ? len2 - h2 - 1 : h2;
    }
    r1 = l1;
    r2 = l2;
}

// Medium entries: entry e = (triangle index into med, outer edge and inner chunk, as in
// medium_inner_chunks).  Lane l takes entry `e` (when `active`): edge x of the triangle's outer pair
// (its direction-0 run, then its direction-1 run).  A pair (x, y) with y on the other
// source-incident pair (the inner one, or the entry's chunk of it) can only complete a triangle
// when |t_y - t_x| <= d13 (d12, d23 <= d13 after normalisation), and on each inner direction list
// those y form one key range (clipped to the window too), found by binary search.  The wavefront then spreads the (x, y) pairs of all its lanes evenly over the lanes
// (pair j belongs to the last lane whose exclusive prefix of pair counts is <= j), so one outer edge
// with many close partners does not stall the others.  Every lane of the wavefront must call this.
// Each pair goes to eval(direction combination 2 d_uv + d_uw, its {v,w} lists, uv key, uw key);
// q gives the window and the d13 of the closeness test.
// With lev (the windowed copies), an entry whose triangle's level is below q.qlev is skipped: that
// triangle is counted by the prefix procedures for this query.  Returns the pairs this wavefront
// evaluated (its share of the visits).
template <class EVAL>
__device__ __forceinline__ uint32_t medium_lanes_eval(const uint32_t *__restrict__ med, const uint32_t *__restrict__ ent,
                                                      uint64_t e, bool active, const uint32_t *__restrict__ eoff,
                                                      const uint64_t *__restrict__ key, const DQuery &q, EVAL &&eval,
                                                      unsigned lane, const uint8_t *__restrict__ lev = nullptr) {
    uint64_t kx = 0;
    uint32_t lo0 = 0, c0 = 0, lo1 = 0, c1 = 0, zb0 = 0, ze0 = 0, zb1 = 0, ze1 = 0, flags = 0;
    if (active && lev && lev[ent[2 * e]] < q.qlev) active = false;
    if (active) {
        const uint32_t t = ent[2 * e], jc = ent[2 * e + 1];
        const uint32_t e_uv = med[3 * (uint64_t)t], e_uw = med[3 * (uint64_t)t + 1], e_vw = med[3 * (uint64_t)t + 2];
        const uint32_t a0 = eoff[2 * e_uv], a1 = eoff[2 * e_uv + 1], a2 = eoff[2 * e_uv + 2];
        const uint32_t b0 = eoff[2 * e_uw], b1 = eoff[2 * e_uw + 1], b2 = eoff[2 * e_uw + 2];
        const bool outer_uv = medium_outer_is_uv(a2 - a0, b2 - b0);
        const uint32_t o0 = outer_uv ? a0 : b0, o1 = outer_uv ? a1 : b1, o2 = outer_uv ? a2 : b2;
        const uint32_t i0 = outer_uv ? b0 : a0, i1 = outer_uv ? b1 : a1, i2 = outer_uv ? b2 : a2;
        // this entry's outer edge and inner chunk [cb, ce): the inner direction runs [i0, i1) and
        // [i1, i2) clipped to it
        const uint32_t nc = medium_inner_chunks(o2 - o0, i2 - i0);
        const uint32_t j = jc / nc, ch = jc - j * nc;
        const uint32_t cb = nc > 1 ? i0 + ch * kInnerChunk : i0;
        const uint32_t ce = nc > 1 && cb + kInnerChunk < i2 ? cb + kInnerChunk : i2;
        const uint32_t r0b = cb < i1 ? cb : i1, r0e = ce < i1 ? ce : i1;
        const uint32_t r1b = cb > i1 ? cb : i1, r1e = ce > i1 ? ce : i1;
        const uint32_t ox = o0 + j;
        flags = (outer_uv ? 1u : 0u) | (ox >= o1 ? 2u : 0u);
        kx = key[ox];
        if (kx >= q.klo && kx < q.khi) {
            const int64_t tx = (int64_t)(kx >> q.shift);
            uint64_t klo = before_time(tx - q.d13, q), khi = before_time(tx + q.d13 + 1, q);
            klo = klo > q.klo ? klo : q.klo;
            khi = khi < q.khi ? khi : q.khi;
            uint32_t hi0, hi1;
            lower2(key, r0b, r0e, klo, khi, lo0, hi0);
            lower2(key, r1b, r1e, klo, khi, lo1, hi1);
            c0 = hi0 - lo0;
            c1 = hi1 - lo1;
            if (c0 + c1) {   // the {v,w} lists, clipped to the window
                zb0 = eoff[2 * e_vw];
                ze0 = eoff[2 * e_vw + 1];
                ze1 = eoff[2 * e_vw + 2];
                zb1 = ze0;
                if (q.windowed) {
                    lower2(key, zb0, ze0, q.klo, q.khi, zb0, ze0);
                    lower2(key, zb1, ze1, q.klo, q.khi, zb1, ze1);
                }
            }
        }
    }
    // exclusive prefix of the lanes' pair counts
    const uint32_t c = c0 + c1;
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= (unsigned)o) incl += y;
    }
    const uint32_t excl = incl - c;
    const uint32_t total = __shfl(incl, 63, 64);
    if (total == 0) return 0;
    const uint32_t kx_lo = (uint32_t)kx, kx_hi = (uint32_t)(kx >> 32);
    for (uint32_t base = 0; base < total; base += 64) {
        const uint32_t jp = base + lane;
        const uint32_t jj = jp < total ? jp : total - 1;
        uint32_t l = 0;   // owner lane of pair jj
#pragma unroll
        for (uint32_t step = 32; step > 0; step >>= 1)
            if (__shfl(excl, l + step, 64) <= jj) l += step;
        const uint32_t r = jj - __shfl(excl, l, 64);
        const uint32_t oc0 = __shfl(c0, l, 64), olo0 = __shfl(lo0, l, 64), olo1 = __shfl(lo1, l, 64);
        const uint32_t ofl = __shfl(flags, l, 64);
        const uint64_t okx = ((uint64_t)(uint32_t)__shfl(kx_hi, l, 64) << 32) | (uint32_t)__shfl(kx_lo, l, 64);
        Lists L;
        L.lo[4] = __shfl(zb0, l, 64);
        L.hi[4] = __shfl(ze0, l, 64);
        L.lo[5] = __shfl(zb1, l, 64);
        L.hi[5] = __shfl(ze1, l, 64);
        if (jp >= total) continue;
        const bool outer_uv = ofl & 1u;
        const uint32_t x_dir = (ofl >> 1) & 1u, y_dir = r < oc0 ? 0u : 1u;
        const uint64_t ky = key[r < oc0 ? olo0 + r : olo1 + (r - oc0)];
        // (uv edge, uw edge) with their directions
        const uint64_t k_uv = outer_uv ? okx : ky, k_uw = outer_uv ? ky : okx;
        const uint32_t d_uv = outer_uv ? x_dir : y_dir, d_uw = outer_uv ? y_dir : x_dir;
        eval(d_uv * 2 + d_uw, L, k_uv, k_uw);
    }
    return total;
}

// one (uv, uw) pair of given direction combination for query q
template <class ACC>
__device__ __forceinline__ void medium_pair_any(int combo, const uint64_t *__restrict__ key, const Lists &L,
                                                const DQuery &q, uint64_t k_uv, uint64_t k_uw, ACC &acc) {
    switch (combo) {
        case 0: medium_pair<0, 0>(key, L, q, k_uv, k_uw, acc); break;
        case 1: medium_pair<0, 1>(key, L, q, k_uv, k_uw, acc); break;
        case 2: medium_pair<1, 0>(key, L, q, k_uv, k_uw, acc); break;
        default: medium_pair<1, 1>(key, L, q, k_uv, k_uw, acc); break;
    }
}

// the medium path for one query into accumulator acc; returns the pairs the wavefront evaluated
template <class ACC>
__device__ __forceinline__ uint32_t medium_lanes(const uint32_t *__restrict__ med, const uint32_t *__restrict__ ent,
                                                 uint64_t e, bool active, const uint32_t *__restrict__ eoff,
                                                 const uint64_t *__restrict__ key, const DQuery &q, ACC &acc,
                                                 unsigned lane, const uint8_t *__restrict__ lev = nullptr) {
    return medium_lanes_eval(med, ent, e, active, eoff, key, q,
                             [&](int combo, const Lists &L, uint64_t k_uv, uint64_t k_uw) {
                                 medium_pair_any(combo, key, L, q, k_uv, k_uw, acc);
                             },
                             lane, lev);
}

// light triangles: P <= light_pair_cap and at most kLightVw edges on {v,w}
constexpr uint64_t kLightVw = 64;

// The unit record of triangle (e_uv, e_uw, e_vw), each pair holding one temporal edge: the edge's
// key sits at eoff[2e] whichever its direction; the direction bit is 1 (towards the earlier vertex
// of u < v < w) when the pair's forward part [eoff[2e], eoff[2e+1]) is empty.
// the record from the three edges' keys and directions (1: head -> tail), pairs uv, uw, vw
__device__ __forceinline__ uint4 unit_record_of(const uint64_t (&k)[3], const int (&dir)[3], int shift) {
    // pairs in key order: first, second, third (0 = uv, 1 = uw, 2 = vw)
    int o0 = 0, o1 = 1, o2 = 2;
    if (k[o1] < k[o0]) { int x = o0; o0 = o1; o1 = x; }
    if (k[o2] < k[o1]) { int x = o1; o1 = o2; o2 = x; }
    if (k[o1] < k[o0]) { int x = o0; o0 = o1; o1 = x; }
    // Figure 3: pi1 (uv, uw, vw), pi2 (uw, uv, vw), pi3 (uv, vw, uw), pi4 (uw, vw, uv),
    // pi5 (vw, uv, uw), pi6 (vw, uw, uv)
    const int pi = o0 == 0 ? (o1 == 1 ? 1 : 3) : (o0 == 1 ? (o1 == 0 ? 2 : 4) : (o1 == 0 ? 5 : 6));
    const int rho = rho_of(dir[0], dir[1], dir[2]);
    const int type = psi_of(pi, rho);
    const uint32_t t1 = (uint32_t)(k[o0] >> shift), t2 = (uint32_t)(k[o1] >> shift),
                   t3 = (uint32_t)(k[o2] >> shift);
    return make_uint4(t1, t2 - t1, t3 - t2, (uint32_t)(((pi - 1) * 8 + (rho - 1)) << 8) | (uint32_t)(type - 1));
}

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
    return unit_record_of(k, dir, shift);
}

// ---------------------------------------------------------------------------------------------
// unit path: one record per triangle with one temporal edge on each pair
// ---------------------------------------------------------------------------------------------
// A query against unit records: the normalised deltas and the window [wlo, whi) as relative times
// (all below 2^31 + 1 on this path; whi = 2^32 - 1 when unwindowed).
struct UQuery {
    uint32_t d12, d23, d13, wlo, whi;
};

inline UQuery unit_query(const DQuery &q) {
    UQuery u;
    u.d12 = (uint32_t)q.d12;
    u.d23 = (uint32_t)q.d23;
    u.d13 = (uint32_t)q.d13;
    u.wlo = q.windowed ? (uint32_t)(q.klo >> q.shift) : 0u;
    u.whi = q.windowed ? (uint32_t)(q.khi >> q.shift) : 0xffffffffu;
    return u;
}

// record r = (t1, t2 - t1, t3 - t2, cell << 8 | type): Definition 1's three delta constraints and
// the window, then one count for its type (or its cell)
template <bool CELLS>
__device__ __forceinline__ void unit_one(const uint4 r, const UQuery &u, uint32_t (&c)[8],
                                         int64_t *__restrict__ cells) {
    const uint32_t g13 = r.y + r.z;
    const bool ok = r.y <= u.d12 && r.z <= u.d23 && g13 <= u.d13 && r.x >= u.wlo && r.x + g13 < u.whi;
    if (CELLS) {
        if (ok) atomicAdd((unsigned long long *)(cells + (r.w >> 8)), 1ull);
    } else {
        const uint32_t ty = r.w & 7u;
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) c[j] += (ok && ty == j) ? 1u : 0u;
    }
}

// records [beg, end) by the BLOCK threads of one workgroup, four loads in flight per thread
template <bool CELLS, unsigned BLOCK>
__device__ __forceinline__ void unit_run(const uint4 *__restrict__ rec, uint64_t beg, uint64_t end,
                                         const UQuery &u, uint32_t (&c)[8], int64_t *__restrict__ cells) {
    uint64_t i = beg + threadIdx.x;
    for (; i + 3 * BLOCK < end; i += 4 * BLOCK) {
        const uint4 r0 = rec[i], r1 = rec[i + BLOCK], r2 = rec[i + 2 * BLOCK], r3 = rec[i + 3 * BLOCK];
        unit_one<CELLS>(r0, u, c, cells);
        unit_one<CELLS>(r1, u, c, cells);
        unit_one<CELLS>(r2, u, c, cells);
        unit_one<CELLS>(r3, u, c, cells);
    }
    for (; i < end; i += BLOCK) unit_one<CELLS>(rec[i], u, c, cells);
}

// XCD-aware block order: blocks are dispatched round-robin over the 8 XCDs, so block b runs on
// XCD b % 8; give each XCD a contiguous range of work so that triangles sharing u (adjacent in
// the list) share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblk) {
    if (nblk % 8) return b;
    return (b % 8) * (nblk / 8) + b / 8;
}

template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// reduce the block's 8 per-lane counters into out8 (block slot of the partials)
template <unsigned BLOCK>
__device__ __forceinline__ void block_store(const int64_t (&t)[8], int64_t *__restrict__ out8) {
    __shared__ int64_t s[BLOCK / 64][8];
    const unsigned wave = threadIdx.x / 64, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int64_t v = wave_sum((long long)t[i]);
        if (lane == 0) s[wave][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        int64_t v = 0;
#pragma unroll
        for (unsigned w = 0; w < BLOCK / 64; ++w) v += s[w][threadIdx.x];
        out8[threadIdx.x] = v;
    }
}

// the 128-bit form: 16 words per block slot, (low, high) per type
template <unsigned BLOCK>
__device__ __forceinline__ void block_store_w(const unsigned __int128 (&t)[8], int64_t *__restrict__ out16) {
    __shared__ unsigned long long s[BLOCK / 64][16];
    const unsigned wave = threadIdx.x / 64, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        unsigned long long lo = (unsigned long long)t[i], hi = (unsigned long long)(t[i] >> 64);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long lo2 = __shfl_xor(lo, o, 64), hi2 = __shfl_xor(hi, o, 64);
            const unsigned long long sum = lo + lo2;
            hi += hi2 + (sum < lo ? 1ull : 0ull);
            lo = sum;
        }
        if (lane == 0) {
            s[wave][2 * i] = lo;
            s[wave][2 * i + 1] = hi;
        }
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        unsigned __int128 v = 0;
#pragma unroll
        for (unsigned w = 0; w < BLOCK / 64; ++w)
            v += ((unsigned __int128)s[w][2 * threadIdx.x + 1] << 64) | s[w][2 * threadIdx.x];
        out16[2 * threadIdx.x] = (int64_t)(uint64_t)v;
        out16[2 * threadIdx.x + 1] = (int64_t)(uint64_t)(v >> 64);
    }
}

// a block's accumulator to its partial slot: 8 words, or 16 in the 128-bit form
template <unsigned BLOCK, class ACC> __device__ __forceinline__ void acc_store(const ACC &acc, int64_t *__restrict__ part,
                                                                              uint64_t slot) {
    block_store<BLOCK>(acc.t, part + 8 * slot);
}
template <unsigned BLOCK> __device__ __forceinline__ void acc_store(const AccW &acc, int64_t *__restrict__ part,
                                                                   uint64_t slot) {
    block_store_w<BLOCK>(acc.t, part + 16 * slot);
}

// add a lane's visits to *visits (when instrumented); every lane of the wavefront must call this
__device__ __forceinline__ void add_visits(unsigned long long *visits, uint64_t v) {
    if (!visits) return;
    const unsigned long long s = wave_sum((unsigned long long)v);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(visits, s);
}

// ---------------------------------------------------------------------------------------------
// heavy path: the prefix-count procedures of Algorithms 1-3
// ---------------------------------------------------------------------------------------------
// A query counts the heavy triangles [hb, n_heavy) (those below its level come first in the list
// order: the suffix is the query's share).  Its scratch indices are relative to that suffix:
// clip[12 (h - hb) + .], prefix slots from hslot[h] - slot_base, chunk totals from the first
// prefix chunk pb.
struct HeavyArgs {
    const uint32_t *heavy, *pchunks, *chunks, *eoff;
    const uint64_t *key, *hslot;
    uint64_t hb, pb, slot_base, ns;   // ns: prefix slots of the suffix (the stride of P's arrays)
    int64_t *P, *T;                   // prefix arrays [kVals][ns]; chunk totals [chunk - pb][kVals]
    uint32_t *clip;                   // clipped bounds of the six lists, 12 words per triangle
    DQuery q;
};

// window-clipped bounds of the six lists of heavy triangle hb + hl
__device__ __forceinline__ void heavy_clip_one(const HeavyArgs &A, uint64_t hl) {
    const uint32_t *t3 = A.heavy + 3 * (A.hb + hl);
    Lists L;
    load_lists(A.eoff, t3[0], t3[1], t3[2], A.key, A.q, L);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        A.clip[12 * hl + 2 * i] = L.lo[i];
        A.clip[12 * hl + 2 * i + 1] = L.hi[i];
    }
}

// full (unclipped) start of the six lists, from the DAG edge offsets
__device__ __forceinline__ void full_lists(const uint32_t *__restrict__ eoff, const uint32_t *__restrict__ t3,
                                           uint32_t (&beg)[7]) {
    // beg[i], beg[i+1] delimit list i for i = 0..3 (uv+, uv-, uw+, uw-)
    beg[0] = eoff[2 * t3[0]];
    beg[1] = eoff[2 * t3[0] + 1];
    beg[2] = eoff[2 * t3[0] + 2];
    beg[3] = eoff[2 * t3[1]];
    beg[4] = eoff[2 * t3[1] + 1];
    beg[5] = eoff[2 * t3[1] + 2];
    beg[6] = 0;
}

// Prefix values per source edge (the cumulative edge counts of Algorithms 1-3), for
// list X of heavy triangle h, against the two vw lists (c = 0, 1):
//   E_c = #{z in vw_c : t_z <= t + d13}                  (Algorithm 1, prefix over S1)
//   A_c = #{z in vw_c : key_z < key}                     (Algorithm 2, prefix over S3)
//   B_c = #{z in vw_c : t_z < t - d23}                   (Algorithm 2, prefix over S3)
//   C_c = #{z in vw_c : t_z < t - d13}                   (Algorithm 3, prefix over S3)
// stored as exclusive prefix sums P_v[r] over the whole list X, r = 0..len(X), where an edge outside
// the window contributes 0 (so P at a clipped position is the clipped list's prefix).
constexpr unsigned kPrefixBlock = 256;
constexpr int kVals = 8;   // E0, E1, A0, A1, B0, B1, C0, C1

template <class T> __device__ __forceinline__ T wave_incl_scan(T v, unsigned lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(v, o, 64);
        if (lane >= (unsigned)o) v += y;
    }
    return v;
}

// A prefix chunk: up to kPrefixBlock consecutive edges of one list X of one heavy triangle,
// pchunks[2 c] = h, pchunks[2 c + 1] = first | X (first, the chunk's offset in the list, is a
// multiple of kPrefixBlock).  Decodes the chunk: its list's full start and length and its slot.
struct PChunk {
    uint32_t h, X, first, fs, len;
    uint64_t slot;   // relative to slot_base
};
__device__ __forceinline__ PChunk pchunk_at(const uint32_t *__restrict__ pchunks, uint64_t c,
                                            const uint32_t *__restrict__ heavy, const uint32_t *__restrict__ eoff,
                                            const uint64_t *__restrict__ hslot, uint64_t slot_base) {
    PChunk k;
    k.h = pchunks[2 * c];
    const uint32_t w = pchunks[2 * c + 1];
    k.X = w & 3u;
    k.first = w & ~(kPrefixBlock - 1);
    uint32_t beg[7];
    full_lists(eoff, heavy + 3 * (uint64_t)k.h, beg);
    const uint32_t len_full[4] = {beg[1] - beg[0], beg[2] - beg[1], beg[4] - beg[3], beg[5] - beg[4]};
    const uint32_t start_full[4] = {beg[0], beg[1], beg[3], beg[4]};
    k.fs = start_full[k.X];
    k.len = len_full[k.X];
    uint64_t slot = hslot[k.h] - slot_base;
    for (uint32_t Y = 0; Y < k.X; ++Y) slot += len_full[Y] + 1;
    k.slot = slot;
    return k;
}

// Phase 1 of the prefix pass, one chunk c by the whole workgroup (kPrefixBlock threads): its edges'
// eight values and their exclusive prefix within the chunk (into P) and the chunk's totals (into
// T).  vis counts the edges inside the window.
__device__ __forceinline__ void heavy_prefix_local_chunk(const HeavyArgs &A, uint64_t c, uint64_t &vis) {
    const unsigned lane = threadIdx.x & 63, wave = threadIdx.x / 64;
    __shared__ int64_t s_tot[kPrefixBlock / 64][kVals];
    const DQuery &q = A.q;
    const uint64_t *key = A.key;
    const PChunk k = pchunk_at(A.pchunks, c, A.heavy, A.eoff, A.hslot, A.slot_base);
    const uint64_t hl = k.h - A.hb;
    const uint32_t lo = A.clip[12 * hl + 2 * k.X], hi = A.clip[12 * hl + 2 * k.X + 1];
    const uint32_t z0 = A.clip[12 * hl + 8], z0e = A.clip[12 * hl + 9];
    const uint32_t z1 = A.clip[12 * hl + 10], z1e = A.clip[12 * hl + 11];
    const uint32_t r = k.first + threadIdx.x;
    const uint32_t p = k.fs + r;
    int64_t v[kVals] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (r < k.len && p >= lo && p < hi) {
        const uint64_t kk = key[p];
        const int64_t t = (int64_t)(kk >> q.shift);
        v[0] = lower(key, z0, z0e, before_time(t + q.d13 + 1, q)) - z0;
        v[1] = lower(key, z1, z1e, before_time(t + q.d13 + 1, q)) - z1;
        v[2] = lower(key, z0, z0e, kk) - z0;
        v[3] = lower(key, z1, z1e, kk) - z1;
        v[4] = lower(key, z0, z0e, before_time(t - q.d23, q)) - z0;
        v[5] = lower(key, z1, z1e, before_time(t - q.d23, q)) - z1;
        v[6] = lower(key, z0, z0e, before_time(t - q.d13, q)) - z0;
        v[7] = lower(key, z1, z1e, before_time(t - q.d13, q)) - z1;
        ++vis;
    }
    int64_t incl[kVals];
#pragma unroll
    for (int i = 0; i < kVals; ++i) incl[i] = wave_incl_scan((long long)v[i], lane);
    if (lane == 63) {
#pragma unroll
        for (int i = 0; i < kVals; ++i) s_tot[wave][i] = incl[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kVals; ++i) {
        int64_t before = 0, total = 0;
        for (unsigned w = 0; w < kPrefixBlock / 64; ++w) {
            if (w < wave) before += s_tot[w][i];
            total += s_tot[w][i];
        }
        if (r < k.len) A.P[(uint64_t)i * A.ns + k.slot + r] = before + incl[i] - v[i];
        if (threadIdx.x == 0) A.T[(c - A.pb) * kVals + i] = total;
    }
    __syncthreads();
}

// Phase 2, one thread per prefix chunk c: a chunk that starts a list walks that list's chunks and
// replaces their totals in T by the exclusive prefix of the totals (each chunk's carry), and writes
// the list's totals at position len of its prefix arrays.
__device__ __forceinline__ void heavy_prefix_scan_list(const HeavyArgs &A, uint64_t c, uint64_t pe) {
    const PChunk k = pchunk_at(A.pchunks, c, A.heavy, A.eoff, A.hslot, A.slot_base);
    if (k.first != 0) return;
    const uint64_t nc = k.len ? (k.len + kPrefixBlock - 1) / kPrefixBlock : 1;
    if (c + nc > pe) return;   // cannot happen: a list's chunks are consecutive
    int64_t run[kVals] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t j = c; j < c + nc; ++j) {
        int64_t *t = A.T + (j - A.pb) * kVals;
#pragma unroll
        for (int i = 0; i < kVals; ++i) {
            const int64_t x = t[i];
            t[i] = run[i];
            run[i] += x;
        }
    }
#pragma unroll
    for (int i = 0; i < kVals; ++i) A.P[(uint64_t)i * A.ns + k.slot + k.len] = run[i];
}

// Phase 3, one chunk c by the whole workgroup: adds its carry to its edges' prefix values.
__device__ __forceinline__ void heavy_prefix_add_chunk(const HeavyArgs &A, uint64_t c) {
    const PChunk k = pchunk_at(A.pchunks, c, A.heavy, A.eoff, A.hslot, A.slot_base);
    const uint32_t r = k.first + threadIdx.x;
    if (r < k.len && k.first > 0) {
        const int64_t *t = A.T + (c - A.pb) * kVals;
#pragma unroll
        for (int i = 0; i < kVals; ++i) A.P[(uint64_t)i * A.ns + k.slot + r] += t[i];
    }
}

// One source edge e (key k, time t) on list X of heavy triangle h, as e2 of Algorithm 1, e1 of
// Algorithm 2 and e2 of Algorithm 3, against both directions of the other source pair (b) and of
// {v,w} (c).
struct HeavyCtx {
    const uint64_t *key;
    const int64_t *P;
    uint64_t n_slots;
    uint64_t slot[4];          // first slot of the prefix arrays of lists 0..3
    uint32_t fs[4];            // full start of lists 0..3 (P is indexed from there)
    uint32_t lo[6], hi[6];     // clipped bounds
};

template <class ACC, int X, int B, int C>
__device__ __forceinline__ void heavy_cell(const HeavyCtx &H, const DQuery &q, uint64_t k, int64_t t,
                                           ACC &acc, const uint32_t (&o)[8]) {
    // element's pair: uv for X = 0, 1 and uw for X = 2, 3; direction a = X & 1
    constexpr bool kUv = X < 2;
    constexpr int a = X & 1;
    constexpr int OL = kUv ? 2 + B : B;            // other source list
    constexpr int DUV = kUv ? a : B, DUW = kUv ? B : a;
    const uint32_t zb = H.lo[4 + C], ze = H.hi[4 + C];
    // searches into the vw list of direction C
    const uint64_t *key = H.key;
    const int64_t r_lt = (int64_t)(lower(key, zb, ze, k) - zb);                          // key < k
    const int64_t r_d23 = (int64_t)(lower(key, zb, ze, before_time(t + q.d23 + 1, q)) - zb); // t <= t + d23
    const int64_t r_d12 = (int64_t)(lower(key, zb, ze, before_time(t + q.d12 + 1, q)) - zb); // t <= t + d12
    const int64_t r_m12 = (int64_t)(lower(key, zb, ze, before_time(t - q.d12, q)) - zb);     // t < t - d12
    const int64_t *P = H.P;
    const uint64_t ns = H.n_slots;
    const uint64_t sb = H.slot[OL] - H.fs[OL];   // P index of absolute position p in list OL: sb + p
    const int64_t *PE = P + (uint64_t)(0 + C) * ns + sb;
    const int64_t *PA = P + (uint64_t)(2 + C) * ns + sb;
    const int64_t *PB = P + (uint64_t)(4 + C) * ns + sb;
    const int64_t *PC = P + (uint64_t)(6 + C) * ns + sb;
    // o[]: searches into the other list (absolute indices), shared by the C = 0, 1 calls
    const uint32_t o_m12 = o[0], o_lt = o[1], o_mid = o[2], o_p12 = o[3], o_p23 = o[4],
                   o_p13 = o[5], o_p1312 = o[6];
    // Algorithm 1 (e = e2 on S2; S1 = other list, S3 = vw_C): pi1 when e is on uw, pi2 on uv
    if (o_lt > o_m12) {
        uint32_t lo1 = o_m12, hi1 = o_lt;
        uint32_t mid = o_mid < lo1 ? lo1 : (o_mid > hi1 ? hi1 : o_mid);
        int64_t c = (PE[mid] - PE[lo1]) - (int64_t)(mid - lo1) * r_lt +
                    (int64_t)(hi1 - mid) * (r_d23 - r_lt);
        if (kUv) acc.template add<Cell<2, DUV, DUW, C>>(c);
        else acc.template add<Cell<1, DUV, DUW, C>>(c);
    }
    // Algorithm 2 (e = e1 on S1; S2 = vw_C, S3 = other list): pi3 when e is on uv, pi4 on uw
    {
        const bool d12_first = q.d12 <= q.d23;
        uint32_t f = o_lt;
        uint32_t x1 = d12_first ? o_p12 : o_p23;
        uint32_t x2 = d12_first ? o_p23 : o_p12;
        x1 = x1 < f ? f : x1;
        x2 = x2 < x1 ? x1 : x2;
        uint32_t x3 = o_p13 < x2 ? x2 : o_p13;
        int64_t c = (PA[x1] - PA[f]) - (int64_t)(x1 - f) * r_lt;
        if (d12_first) c += (int64_t)(x2 - x1) * (r_d12 - r_lt);
        else c += (PA[x2] - PA[x1]) - (PB[x2] - PB[x1]);
        c += (int64_t)(x3 - x2) * r_d12 - (PB[x3] - PB[x2]);
        if (kUv) acc.template add<Cell<3, DUV, DUW, C>>(c);
        else acc.template add<Cell<4, DUV, DUW, C>>(c);
    }
    // Algorithm 3 (e = e2 on S2; S3 = other list, S1 = vw_C): pi5 when e is on uv, pi6 on uw
    {
        uint32_t f = o_lt;
        uint32_t s = o_p1312 < f ? f : o_p1312;
        uint32_t e = o_p23 < s ? s : o_p23;
        int64_t c = (int64_t)(s - f) * (r_lt - r_m12) + (int64_t)(e - s) * r_lt - (PC[e] - PC[s]);
        if (kUv) acc.template add<Cell<5, DUV, DUW, C>>(c);
        else acc.template add<Cell<6, DUV, DUW, C>>(c);
    }
}

template <class ACC, int X, int B>
__device__ __forceinline__ void heavy_other(const HeavyCtx &H, const DQuery &q, uint64_t k, int64_t t,
                                            ACC &acc) {
    constexpr int OL = X < 2 ? 2 + B : B;
    const uint32_t ob = H.lo[OL], oe = H.hi[OL];
    const uint64_t *key = H.key;
    uint32_t o[8];
    o[0] = lower(key, ob, oe, before_time(t - q.d12, q));              // t < t - d12
    o[1] = lower(key, ob, oe, k);                                     // key < k
    o[2] = lower(key, ob, oe, before_time(t - q.d13 + q.d23 + 1, q)); // t <= t - d13 + d23
    o[3] = lower(key, ob, oe, before_time(t + q.d12 + 1, q));         // t <= t + d12
    o[4] = lower(key, ob, oe, before_time(t + q.d23 + 1, q));         // t <= t + d23
    o[5] = lower(key, ob, oe, before_time(t + q.d13 + 1, q));         // t <= t + d13
    o[6] = lower(key, ob, oe, before_time(t + q.d13 - q.d12 + 1, q)); // t <= t + d13 - d12
    o[7] = 0;
    heavy_cell<ACC, X, B, 0>(H, q, k, t, acc, o);
    heavy_cell<ACC, X, B, 1>(H, q, k, t, acc, o);
}

template <class ACC, int X>
__device__ __forceinline__ void heavy_elem(const HeavyCtx &H, const DQuery &q, uint32_t p, ACC &acc) {
    const uint64_t k = H.key[p];
    const int64_t t = (int64_t)(k >> q.shift);
    heavy_other<ACC, X, 0>(H, q, k, t, acc);
    heavy_other<ACC, X, 1>(H, q, k, t, acc);
}

// The count pass for one chunk ch (256 source edges of the four lists in a row), one edge per
// thread of a 256-thread workgroup, into acc.
template <class ACC>
__device__ __forceinline__ void heavy_count_chunk(const HeavyArgs &A, uint64_t ch, ACC &acc) {
    const uint32_t h = A.chunks[2 * ch], first = A.chunks[2 * ch + 1];
    const uint64_t hl = h - A.hb;
    const uint32_t *t3 = A.heavy + 3 * (uint64_t)h;
    uint32_t beg[7];
    full_lists(A.eoff, t3, beg);
    const uint32_t len_full[4] = {beg[1] - beg[0], beg[2] - beg[1], beg[4] - beg[3], beg[5] - beg[4]};
    const uint32_t start_full[4] = {beg[0], beg[1], beg[3], beg[4]};
    HeavyCtx H;
    H.key = A.key;
    H.P = A.P;
    H.n_slots = A.ns;
    uint64_t s = A.hslot[h] - A.slot_base;
#pragma unroll
    for (int Y = 0; Y < 4; ++Y) {
        H.slot[Y] = s;
        H.fs[Y] = start_full[Y];
        s += len_full[Y] + 1;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        H.lo[i] = A.clip[12 * hl + 2 * i];
        H.hi[i] = A.clip[12 * hl + 2 * i + 1];
    }
    uint32_t ei = first + threadIdx.x;
    const uint32_t total = len_full[0] + len_full[1] + len_full[2] + len_full[3];
    if (ei < total) {
        int X = 0;
        while (ei >= len_full[X]) {
            ei -= len_full[X];
            ++X;
        }
        const uint32_t p = start_full[X] + ei;
        if (p >= H.lo[X] && p < H.hi[X]) {
            ++acc.visits;
            switch (X) {
                case 0: heavy_elem<ACC, 0>(H, A.q, p, acc); break;
                case 1: heavy_elem<ACC, 1>(H, A.q, p, acc); break;
                case 2: heavy_elem<ACC, 2>(H, A.q, p, acc); break;
                default: heavy_elem<ACC, 3>(H, A.q, p, acc); break;
            }
        }
    }
}

}  // namespace cdev
}  // namespace dt
