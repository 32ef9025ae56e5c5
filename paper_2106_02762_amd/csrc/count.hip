// Per-triangle temporal counting (Algorithm 4 with Algorithms 1-3, Section 5 and Appendix A) and
// the per-type reduction.
//
// Every static triangle <u, v, w> (u first in the degeneracy ordering, v before w) owns six
// key-sorted edge lists: uv+ (u->v), uv- (v->u), uw+, uw-, vw+, vw-.  A cell (pi, rho) of the
// paper is an ordering pi (Figure 3) and one direction per pair rho (Figure 4); its count goes to
// type psi(pi, rho) (Table 2).  Only the lists on the two pairs at u are ever walked; the {v,w}
// lists are only searched (Section 5, "source vertex").
//
// Paths, chosen per triangle by the scheduler:
//  - unit: a triangle with one temporal edge on each pair has its ordering, orientation and type
//    fixed at build time; a query tests the record's three times against its deltas and window
//    (Definition 1) and adds one to that type.  A pure stream of 16-byte records.
//  - light: one lane walks every pair (x, y) of edges from the uv and uw lists (the pairwise form
//    of Lemma 1).  With x, y fixed and ordered, the third edge z on {v,w} is first, middle or last,
//    and each case is one key range of the vw list found by binary search; that is cells
//    (pi5|pi6), (pi3|pi4) and (pi1|pi2) respectively.
//  - medium: one lane per edge x of the triangle's smaller source-incident pair; only the edges y
//    of the other pair within d13 of x can complete a triangle, so the lane finds those by binary
//    search, and each wavefront spreads the (x, y) pairs of its lanes evenly over them, each pair
//    then handled as on the light path.
//  - heavy: the prefix-count procedures.  For every edge on a uv or uw list a prefix pass stores
//    the cumulative counts that Algorithms 1-3 need (CEC of Section 5), and a second pass walks
//    the same edges as e2 (Algorithm 1: pi1/pi2), e1 (Algorithm 2: pi3/pi4) and e2 (Algorithm 3:
//    pi5/pi6), each with a constant number of binary searches, split into chunks across
//    workgroups.  The formulas are the paper's, restated for keys (t, input index) so that equal
//    timestamps are handled, with the region bounds written as max/min clamps.
//
// A query with a time window walks the windowed copies of the light and medium lists, ordered by
// window cell, and only the cells that can hold a triangle inside its window (the unit records by
// their first time likewise).
//
// Counts are int64 and summed per lane, per wave, per block, then per launch, with no atomics on
// the result (cells mode, a diagnostic, uses atomics).
#include "count_dev.h"

namespace dt {

using namespace cdev;

namespace {

template <bool CELLS, unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_light(Ranges R, const uint32_t *__restrict__ tri, const uint32_t *__restrict__ eoff,
        const uint64_t *__restrict__ key, DQuery q, int64_t *__restrict__ partial,
        int64_t *__restrict__ cells) {
    Acc<CELLS> acc;
    acc.cells = cells;
    const uint64_t n_tri = R.pre[R.n];
    const uint32_t nblk = gridDim.x;
    const uint32_t b = xcd_block(blockIdx.x, nblk);
    const uint64_t per = (n_tri + nblk - 1) / nblk;
    const uint64_t beg = (uint64_t)b * per;
    const uint64_t end = beg + per < n_tri ? beg + per : n_tri;
    uint32_t r = 0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += BLOCK)
        light_tri(tri, range_at(R, r, i), eoff, key, q, acc);
    if (!CELLS) block_store<BLOCK>(acc.t, partial + 8 * (uint64_t)blockIdx.x);
}

// medium path: wave w takes the 64 entries from 64 w on, then those from 64 (w + W) on, ...
template <bool CELLS, unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_medium(Ranges R, const uint32_t *__restrict__ med, const uint32_t *__restrict__ ent,
         const uint32_t *__restrict__ eoff, const uint64_t *__restrict__ key, DQuery q,
         int64_t *__restrict__ partial, int64_t *__restrict__ cells) {
    Acc<CELLS> acc;
    acc.cells = cells;
    const unsigned lane = threadIdx.x & 63;
    const uint64_t n_ent = R.pre[R.n];
    const uint64_t W = (uint64_t)gridDim.x * (BLOCK / 64);
    uint32_t r = 0;
    for (uint64_t b = ((uint64_t)blockIdx.x * (BLOCK / 64) + threadIdx.x / 64) * 64; b < n_ent; b += W * 64) {
        const uint64_t j = b + lane;
        const bool active = j < n_ent;
        medium_lanes(med, ent, active ? range_at(R, r, j) : 0, active, eoff, key, q, acc, lane);
    }
    if (!CELLS) block_store<BLOCK>(acc.t, partial + 8 * (uint64_t)blockIdx.x);
}

// unit path: block b takes a contiguous run of the records [beg, end)
template <bool CELLS, unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_unit(uint64_t beg, uint64_t end, const uint4 *__restrict__ rec, UQuery u, int64_t *__restrict__ partial,
       int64_t *__restrict__ cells) {
    const uint64_t n = end - beg;
    const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b = beg + (uint64_t)blockIdx.x * per;
    const uint64_t e = b + per < end ? b + per : end;
    uint32_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (b < e) unit_run<CELLS, BLOCK>(rec, b, e, u, c, cells);
    if (!CELLS) {
        int64_t t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) t[j] = c[j];
        block_store<BLOCK>(t, partial + 8 * (uint64_t)blockIdx.x);
    }
}

// ---------------------------------------------------------------------------------------------
// heavy path
// ---------------------------------------------------------------------------------------------
// window-clipped bounds of the six lists of every heavy triangle
__global__ void k_heavy_clip(uint64_t n_heavy, const uint32_t *__restrict__ tri,
                             const uint32_t *__restrict__ eoff, const uint64_t *__restrict__ key,
                             DQuery q, uint32_t *__restrict__ clip) {
    uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n_heavy) return;
    Lists L;
    load_lists(eoff, tri[3 * h], tri[3 * h + 1], tri[3 * h + 2], key, q, L);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        clip[12 * h + 2 * i] = L.lo[i];
        clip[12 * h + 2 * i + 1] = L.hi[i];
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
// stored as exclusive prefix sums P_v[r] over the clipped list, r = 0..len.
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

__global__ void __launch_bounds__(kPrefixBlock)
k_heavy_prefix(uint64_t n_heavy, const uint32_t *__restrict__ tri, const uint32_t *__restrict__ eoff,
               const uint64_t *__restrict__ key, const uint32_t *__restrict__ clip,
               const uint64_t *__restrict__ hslot, uint64_t n_slots, DQuery q,
               int64_t *__restrict__ P) {
    const uint64_t h = blockIdx.x / 4;
    const int X = blockIdx.x % 4;
    if (h >= n_heavy) return;
    const uint32_t *t3 = tri + 3 * h;
    uint32_t beg[7];
    full_lists(eoff, t3, beg);
    // slots of the four source lists follow each other, sized by the unclipped lengths
    const uint32_t len_full[4] = {beg[1] - beg[0], beg[2] - beg[1], beg[4] - beg[3], beg[5] - beg[4]};
    uint64_t base = hslot[h];
    for (int Y = 0; Y < X; ++Y) base += len_full[Y] + 1;
    const uint32_t lo = clip[12 * h + 2 * X], hi = clip[12 * h + 2 * X + 1];
    const uint32_t z0 = clip[12 * h + 8], z0e = clip[12 * h + 9];
    const uint32_t z1 = clip[12 * h + 10], z1e = clip[12 * h + 11];
    const uint32_t len = hi - lo;
    const unsigned lane = threadIdx.x & 63, wave = threadIdx.x / 64;
    __shared__ int64_t s_tot[kPrefixBlock / 64][kVals];
    int64_t carry[kVals] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t c0 = 0; c0 < len; c0 += kPrefixBlock) {
        const uint32_t r = c0 + threadIdx.x;
        int64_t v[kVals] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (r < len) {
            const uint64_t k = key[lo + r];
            const int64_t t = (int64_t)(k >> q.shift);
            v[0] = lower(key, z0, z0e, before_time(t + q.d13 + 1, q)) - z0;
            v[1] = lower(key, z1, z1e, before_time(t + q.d13 + 1, q)) - z1;
            v[2] = lower(key, z0, z0e, k) - z0;
            v[3] = lower(key, z1, z1e, k) - z1;
            v[4] = lower(key, z0, z0e, before_time(t - q.d23, q)) - z0;
            v[5] = lower(key, z1, z1e, before_time(t - q.d23, q)) - z1;
            v[6] = lower(key, z0, z0e, before_time(t - q.d13, q)) - z0;
            v[7] = lower(key, z1, z1e, before_time(t - q.d13, q)) - z1;
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
            int64_t before = carry[i];
            int64_t total = 0;
            for (unsigned w = 0; w < kPrefixBlock / 64; ++w) {
                if (w < wave) before += s_tot[w][i];
                total += s_tot[w][i];
            }
            if (r < len) P[(uint64_t)i * n_slots + base + r] = before + incl[i] - v[i];
            carry[i] += total;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kVals; ++i) P[(uint64_t)i * n_slots + base + len] = carry[i];
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
    uint32_t lo[6], hi[6];     // clipped bounds
};

template <bool CELLS, int X, int B, int C>
__device__ __forceinline__ void heavy_cell(const HeavyCtx &H, const DQuery &q, uint64_t k, int64_t t,
                                           Acc<CELLS> &acc, const uint32_t (&o)[8]) {
    // element's pair: uv for X = 0, 1 and uw for X = 2, 3; direction a = X & 1
    constexpr bool kUv = X < 2;
    constexpr int a = X & 1;
    constexpr int OL = kUv ? 2 + B : B;            // other source list
    constexpr int DUV = kUv ? a : B, DUW = kUv ? B : a;
    const uint32_t zb = H.lo[4 + C], ze = H.hi[4 + C];
    const uint32_t olo = H.lo[OL];
    // searches into the vw list of direction C
    const uint64_t *key = H.key;
    const int64_t r_lt = (int64_t)(lower(key, zb, ze, k) - zb);                          // key < k
    const int64_t r_d23 = (int64_t)(lower(key, zb, ze, before_time(t + q.d23 + 1, q)) - zb); // t <= t + d23
    const int64_t r_d12 = (int64_t)(lower(key, zb, ze, before_time(t + q.d12 + 1, q)) - zb); // t <= t + d12
    const int64_t r_m12 = (int64_t)(lower(key, zb, ze, before_time(t - q.d12, q)) - zb);     // t < t - d12
    const int64_t *P = H.P;
    const uint64_t ns = H.n_slots;
    const uint64_t sb = H.slot[OL] - olo;   // P index of absolute position p in list OL: sb + p
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

template <bool CELLS, int X, int B>
__device__ __forceinline__ void heavy_other(const HeavyCtx &H, const DQuery &q, uint64_t k, int64_t t,
                                            Acc<CELLS> &acc) {
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
    heavy_cell<CELLS, X, B, 0>(H, q, k, t, acc, o);
    heavy_cell<CELLS, X, B, 1>(H, q, k, t, acc, o);
}

template <bool CELLS, int X>
__device__ __forceinline__ void heavy_elem(const HeavyCtx &H, const DQuery &q, uint32_t p,
                                           Acc<CELLS> &acc) {
    const uint64_t k = H.key[p];
    const int64_t t = (int64_t)(k >> q.shift);
    heavy_other<CELLS, X, 0>(H, q, k, t, acc);
    heavy_other<CELLS, X, 1>(H, q, k, t, acc);
}

template <bool CELLS, unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_heavy_count(uint64_t n_chunks, const uint32_t *__restrict__ chunks, const uint32_t *__restrict__ tri,
              const uint32_t *__restrict__ eoff, const uint64_t *__restrict__ key,
              const uint32_t *__restrict__ clip, const uint64_t *__restrict__ hslot,
              uint64_t n_slots, const int64_t *__restrict__ P, DQuery q,
              int64_t *__restrict__ partial, int64_t *__restrict__ cells) {
    Acc<CELLS> acc;
    acc.cells = cells;
    for (uint64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
        const uint32_t h = chunks[2 * ch], first = chunks[2 * ch + 1];
        const uint32_t *t3 = tri + 3 * (uint64_t)h;
        uint32_t beg[7];
        full_lists(eoff, t3, beg);
        const uint32_t len_full[4] = {beg[1] - beg[0], beg[2] - beg[1], beg[4] - beg[3], beg[5] - beg[4]};
        const uint32_t start_full[4] = {beg[0], beg[1], beg[3], beg[4]};
        HeavyCtx H;
        H.key = key;
        H.P = P;
        H.n_slots = n_slots;
        uint64_t s = hslot[h];
#pragma unroll
        for (int Y = 0; Y < 4; ++Y) {
            H.slot[Y] = s;
            s += len_full[Y] + 1;
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            H.lo[i] = clip[12 * (uint64_t)h + 2 * i];
            H.hi[i] = clip[12 * (uint64_t)h + 2 * i + 1];
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
                switch (X) {
                    case 0: heavy_elem<CELLS, 0>(H, q, p, acc); break;
                    case 1: heavy_elem<CELLS, 1>(H, q, p, acc); break;
                    case 2: heavy_elem<CELLS, 2>(H, q, p, acc); break;
                    default: heavy_elem<CELLS, 3>(H, q, p, acc); break;
                }
            }
        }
    }
    if (!CELLS) block_store<BLOCK>(acc.t, partial + 8 * (uint64_t)blockIdx.x);
}

// final reduction of the per-block partials into out8 (deterministic order)
__global__ void __launch_bounds__(256)
k_reduce(uint64_t n_part, const int64_t *__restrict__ partial, int64_t *__restrict__ out8) {
    int64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t i = threadIdx.x; i < n_part; i += 256) {
#pragma unroll
        for (int j = 0; j < 8; ++j) t[j] += partial[8 * i + j];
    }
    block_store<256>(t, out8);
}

__global__ void k_zero(uint64_t n, int64_t *__restrict__ p) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------------------------
// sweeps: several delta triples (one window) per visit of the triangle data
// ---------------------------------------------------------------------------------------------
struct SweepQ {
    DQuery q[kSweepMax];
    UQuery u[kSweepMax];
    uint32_t k;
    int64_t d13max;   // largest d13 of the k triples
};

// adds a sweep's contributions to one triple's eight LDS counters (of this wavefront)
struct AccSweep {
    unsigned long long *s;
    template <class CA, class CB> __device__ __forceinline__ void add2(bool first, int64_t v) {
        if (v) atomicAdd(&s[first ? CA::type : CB::type], (unsigned long long)v);
    }
    template <class C> __device__ __forceinline__ void add(int64_t v) {
        if (v) atomicAdd(&s[C::type], (unsigned long long)v);
    }
};

// The (uv, uw) pairs of one light triangle's direction lists A, B, each tested against every
// triple: the enumeration and the keys are shared, the searches that depend on the deltas are not.
template <int A, int B>
__device__ __forceinline__ void light_pairs_sweep(const uint64_t *__restrict__ key, const Lists &L, const SweepQ &Q,
                                                  unsigned long long *sw) {
    const uint32_t xb = L.lo[A], xe = L.hi[A], yb = L.lo[2 + B], ye = L.hi[2 + B];
    const int shift = Q.q[0].shift;
    for (uint32_t ix = xb; ix < xe; ++ix) {
        const uint64_t kx = key[ix];
        for (uint32_t iy = yb; iy < ye; ++iy) {
            const uint64_t ky = key[iy];
            const bool uv_first = kx < ky;
            const uint64_t k_lo = uv_first ? kx : ky, k_hi = uv_first ? ky : kx;
            const int64_t t_lo = (int64_t)(k_lo >> shift), t_hi = (int64_t)(k_hi >> shift);
            const int64_t gap = t_hi - t_lo;
            if (gap > Q.d13max) continue;
            for (uint32_t j = 0; j < Q.k; ++j) {
                const DQuery &q = Q.q[j];
                if (gap > q.d13) continue;
                AccSweep a{sw + 8 * j};
                light_third<A, B, 0>(key, L, q, uv_first, k_lo, k_hi, t_lo, t_hi, gap, a);
                light_third<A, B, 1>(key, L, q, uv_first, k_lo, k_hi, t_lo, t_hi, gap, a);
            }
        }
    }
}

// a block's sweep counters (per wavefront, [8 j + type]) to its partial slots
template <unsigned BLOCK>
__device__ __forceinline__ void sweep_flush(unsigned long long (*s_sw)[kSweepMax * 8], uint32_t k,
                                            int64_t *__restrict__ part, uint64_t slot) {
    __syncthreads();
    if (threadIdx.x < 8 * k) {
        unsigned long long v = 0;
#pragma unroll
        for (unsigned w = 0; w < BLOCK / 64; ++w) v += s_sw[w][threadIdx.x];
        part[8 * (slot * k + threadIdx.x / 8) + threadIdx.x % 8] = (int64_t)v;
    }
}

// unit records: each record is read once and tested against every delta triple.  A wavefront
// takes 64 records at a time; for each triple the lanes' pass/fail bits form one 64-bit ballot, as
// do the lanes of each type.  Lane l keeps the wavefront's count of (triple l / 8, type l % 8): it
// adds the popcount of that triple's ballot masked by that type's ballot.
template <unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_unit_sweep(uint64_t beg, uint64_t end, const uint4 *__restrict__ rec, SweepQ Q, int64_t *__restrict__ part,
             uint64_t slot0) {
    static_assert(kSweepMax * 8 == 64, "one counter per lane");
    __shared__ uint32_t s_cnt[BLOCK / 64][64];
    const unsigned lane = threadIdx.x & 63, wave = threadIdx.x / 64;
    const uint32_t my_j = lane >> 3, my_t = lane & 7;
    const uint64_t n = end - beg;
    const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b = beg + (uint64_t)blockIdx.x * per;
    const uint64_t e = b + per < end ? b + per : end;
    uint32_t cnt = 0;
    // the window is the same for every triple: test it once per record
    const uint32_t wlo = Q.u[0].wlo, whi = Q.u[0].whi;
    auto test = [&](const uint4 r, bool valid) {
        const uint32_t g13 = r.y + r.z, ty = r.w & 7u;
        valid = valid && r.x >= wlo && r.x + g13 < whi;
        uint64_t tsel = 0, jsel = 0;
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t) {
            const uint64_t m = __ballot(valid && ty == t);
            tsel = my_t == t ? m : tsel;
        }
#pragma unroll
        for (uint32_t j = 0; j < kSweepMax; ++j) {
            if (j < Q.k) {
                const UQuery &u = Q.u[j];
                const uint64_t m = __ballot(valid && r.y <= u.d12 && r.z <= u.d23 && g13 <= u.d13);
                jsel = my_j == j ? m : jsel;
            }
        }
        cnt += (uint32_t)__popcll(jsel & tsel);
    };
    // two records per lane in flight; the loop bounds are the same for the whole wavefront
    uint64_t base = b + 64 * wave;
    for (; base + BLOCK < e; base += 2 * BLOCK) {
        const uint64_t i0 = base + lane, i1 = base + BLOCK + lane;
        const bool v1 = i1 < e;
        const uint4 r0 = rec[i0];
        const uint4 r1 = v1 ? rec[i1] : make_uint4(0u, 0u, 0u, 0u);
        test(r0, true);
        test(r1, v1);
    }
    if (base < e) {
        const uint64_t i0 = base + lane;
        const bool v0 = i0 < e;
        test(v0 ? rec[i0] : make_uint4(0u, 0u, 0u, 0u), v0);
    }
    s_cnt[wave][lane] = cnt;
    __syncthreads();
    if (threadIdx.x < 8 * Q.k) {
        int64_t v = 0;
#pragma unroll
        for (unsigned w = 0; w < BLOCK / 64; ++w) v += s_cnt[w][threadIdx.x];
        part[8 * ((slot0 + blockIdx.x) * Q.k + threadIdx.x / 8) + threadIdx.x % 8] = v;
    }
}

// light triangles: each lane's triangles once, every pair tested against every triple
template <unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_light_sweep(Ranges R, const uint32_t *__restrict__ tri, const uint32_t *__restrict__ eoff,
              const uint64_t *__restrict__ key, SweepQ Q, int64_t *__restrict__ part, uint64_t slot0) {
    __shared__ unsigned long long s_sw[BLOCK / 64][kSweepMax * 8];
    for (unsigned x = threadIdx.x; x < (BLOCK / 64) * kSweepMax * 8; x += BLOCK) (&s_sw[0][0])[x] = 0;
    __syncthreads();
    unsigned long long *sw = s_sw[threadIdx.x / 64];
    const uint64_t n_tri = R.pre[R.n];
    const uint32_t nblk = gridDim.x;
    const uint32_t b = xcd_block(blockIdx.x, nblk);
    const uint64_t per = (n_tri + nblk - 1) / nblk;
    const uint64_t beg = (uint64_t)b * per;
    const uint64_t end = beg + per < n_tri ? beg + per : n_tri;
    uint32_t r = 0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += BLOCK) {
        const uint64_t t = range_at(R, r, i);
        Lists L;
        load_lists(eoff, tri[3 * t], tri[3 * t + 1], tri[3 * t + 2], key, Q.q[0], L);   // one window
        light_pairs_sweep<0, 0>(key, L, Q, sw);
        light_pairs_sweep<0, 1>(key, L, Q, sw);
        light_pairs_sweep<1, 0>(key, L, Q, sw);
        light_pairs_sweep<1, 1>(key, L, Q, sw);
    }
    sweep_flush<BLOCK>(s_sw, Q.k, part, slot0 + blockIdx.x);
}

// medium entries: each entry's close pairs found once, for the largest d13 of the triples, and
// every pair tested against every triple
template <unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_medium_sweep(Ranges R, const uint32_t *__restrict__ med, const uint32_t *__restrict__ ent,
               const uint32_t *__restrict__ eoff, const uint64_t *__restrict__ key, SweepQ Q,
               int64_t *__restrict__ part, uint64_t slot0) {
    __shared__ unsigned long long s_sw[BLOCK / 64][kSweepMax * 8];
    for (unsigned x = threadIdx.x; x < (BLOCK / 64) * kSweepMax * 8; x += BLOCK) (&s_sw[0][0])[x] = 0;
    __syncthreads();
    unsigned long long *sw = s_sw[threadIdx.x / 64];
    const unsigned lane = threadIdx.x & 63;
    const uint64_t n_ent = R.pre[R.n];
    const uint64_t W = (uint64_t)gridDim.x * (BLOCK / 64);
    DQuery qr = Q.q[0];   // the window, and the widest closeness
    qr.d13 = Q.d13max;
    uint32_t r = 0;
    for (uint64_t b = ((uint64_t)blockIdx.x * (BLOCK / 64) + threadIdx.x / 64) * 64; b < n_ent; b += W * 64) {
        const uint64_t x = b + lane;
        const bool active = x < n_ent;
        medium_lanes_eval(med, ent, active ? range_at(R, r, x) : 0, active, eoff, key, qr,
                          [&](int combo, const Lists &L, uint64_t k_uv, uint64_t k_uw) {
                              for (uint32_t j = 0; j < Q.k; ++j) {
                                  AccSweep a{sw + 8 * j};
                                  medium_pair_any(combo, key, L, Q.q[j], k_uv, k_uw, a);
                              }
                          },
                          lane);
    }
    sweep_flush<BLOCK>(s_sw, Q.k, part, slot0 + blockIdx.x);
}

// out[8 j + i] (+)= sum over slots of part[8 (K slot + j) + i]; block j for query j
__global__ void __launch_bounds__(256)
k_reduce_sweep(uint64_t n_slot, uint32_t k, const int64_t *__restrict__ part, int64_t *__restrict__ out, int add) {
    const uint32_t j = blockIdx.x;
    int64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t i = threadIdx.x; i < n_slot; i += 256) {
#pragma unroll
        for (int x = 0; x < 8; ++x) t[x] += part[8 * (i * k + j) + x];
    }
    __shared__ int64_t s_prev[8];
    if (threadIdx.x < 8) s_prev[threadIdx.x] = add ? out[8 * j + threadIdx.x] : 0;
    __syncthreads();
    block_store<256>(t, out + 8 * j);
    __syncthreads();
    if (threadIdx.x < 8) out[8 * j + threadIdx.x] += s_prev[threadIdx.x];
}

constexpr unsigned kLightBlock = 256;
constexpr unsigned kUnitBlock = 256;
constexpr uint64_t kUnitPerBlock = 16384;   // records per workgroup at least (64 per thread)

}  // namespace

int normalise_query(const dt_graph *g, const dt_query *qq, DQuery *out, bool *empty) {
    if (!qq) return fail(DT_EINVAL, "null query");
    if (qq->d13 < 0 || qq->d12 < 0 || qq->d23 < 0)
        return fail(DT_EINVAL, "deltas must be >= 0 (got %lld, %lld, %lld)", (long long)qq->d13,
                    (long long)qq->d12, (long long)qq->d23);
    if (qq->t_lo > qq->t_hi) return fail(DT_EINVAL, "window t_lo > t_hi");
    DQuery q{};
    const int64_t span = g->span;
    auto clampd = [&](int64_t d) { return d > span ? span : d; };
    int64_t d13 = clampd(qq->d13), d12 = clampd(qq->d12), d23 = clampd(qq->d23);
    // the same constraint set: t2-t1 <= t3-t1 and t3-t2 <= t3-t1, and t3-t1 = (t3-t2)+(t2-t1)
    d12 = d12 < d13 ? d12 : d13;
    d23 = d23 < d13 ? d23 : d13;
    d13 = d13 < d12 + d23 ? d13 : d12 + d23;
    q.d13 = d13;
    q.d12 = d12;
    q.d23 = d23;
    q.span = span;
    q.shift = g->shift;
    *empty = (g->m == 0);
    if (qq->t_lo <= g->t_min && qq->t_hi >= g->t_max) {
        q.windowed = 0;
        q.klo = 0;
        q.khi = ~0ull;
    } else {
        q.windowed = 1;
        if (qq->t_hi < g->t_min || qq->t_lo > g->t_max) {
            *empty = true;
            q.klo = q.khi = 0;
        } else {
            int64_t lo = qq->t_lo < g->t_min ? 0 : qq->t_lo - g->t_min;
            int64_t hi = qq->t_hi > g->t_max ? span : qq->t_hi - g->t_min;   // inclusive
            q.klo = (uint64_t)lo << g->shift;
            q.khi = (uint64_t)(hi + 1) << g->shift;
        }
    }
    *out = q;
    return DT_OK;
}

void count_plan(const dt_graph *g, const DQuery &q, unsigned parts, CountPlan &p) {
    const dt_ctx *ctx = g->ctx;
    const Schedule &S = g->sched;
    p.parts = parts;
    const bool do_light = parts & 1, do_medium = parts & 2, do_heavy = parts & 4;
    // the parts of the light and medium lists a windowed query can see
    cell_ranges(S.light_cells, S.cell_shift, q, p.lr);
    cell_ranges(S.mitem_cells, S.cell_shift, q, p.mr);
    const uint64_t nl = p.lr.pre[p.lr.n], nmi = p.mr.pre[p.mr.n];
    p.light = (q.windowed ? S.light_w : S.light).as<uint32_t>();
    p.medium = (q.windowed ? S.medium_w : S.medium).as<uint32_t>();
    p.mitems = (q.windowed ? S.mitems_w : S.mitems).as<uint32_t>();
    const unsigned light_grid = (nl && do_light) ? (unsigned)std::min<uint64_t>(
        (nl + kLightBlock - 1) / kLightBlock, (uint64_t)ctx->num_cus * 16) : 0;
    p.lg = light_grid ? ((light_grid + 7) / 8) * 8 : 0;
    p.hg = (S.n_chunks && do_heavy) ? (unsigned)std::min<uint64_t>(S.n_chunks, (uint64_t)ctx->num_cus * 16) : 0;
    p.mg = (nmi && do_medium) ? (unsigned)std::min<uint64_t>((nmi + 255) / 256, (uint64_t)ctx->num_cus * 8) : 0;
    p.ub = p.ue = 0;
    if (S.n_unit && (parts & 8)) unit_range(g, q, &p.ub, &p.ue);
    p.ug = p.ue > p.ub ? (unsigned)std::min<uint64_t>((p.ue - p.ub + kUnitPerBlock - 1) / kUnitPerBlock,
                                                      (uint64_t)ctx->num_cus * 8) : 0;
    p.n_part = (uint64_t)p.lg + p.hg + p.mg + p.ug;
    p.part_bytes = (p.n_part + 1) * 8 * sizeof(int64_t);
    p.heavy_bytes = (S.n_heavy && do_heavy) ? S.n_slots * kVals * sizeof(int64_t) + 12 * 4 * S.n_heavy + 256 : 0;
}

// Enqueue one planned count on stream s: partials -> out8_dev (int64[8]); cells mode accumulates the
// 48 cells into cells_dev (zeroed here) instead.  The scratch must hold the plan's needs.
int count_launch(dt_graph *g, const DQuery &q, const CountPlan &p, int64_t *out8_dev, hipStream_t s, bool cells,
                 int64_t *cells_dev, const ScratchView &sv) {
    dt_ctx *ctx = g->ctx;
    Schedule &S = g->sched;
    if (sv.part_bytes < p.part_bytes || sv.heavy_bytes < p.heavy_bytes)
        return fail(DT_EINVAL, "count scratch too small (%zu of %zu, %zu of %zu bytes)", sv.part_bytes, p.part_bytes,
                    sv.heavy_bytes, p.heavy_bytes);
    const unsigned lg = p.lg, hg = p.hg, mg = p.mg, ug = p.ug;
    const uint64_t n_part = p.n_part;
    int64_t *part = sv.part;
    if (cells) {
        k_zero<<<1, 64, 0, s>>>(48, cells_dev);
        DT_HIP(hipGetLastError());
    }
    // The light and medium kernels are independent of the unit and heavy ones (each writes its own
    // partial slots): when more than one path has work, they run on the context's side streams,
    // forked from s here and joined back before the reduction, so their latency-bound tails overlap.
    hipStream_t sl = s, sm = s;
    const bool fork = ctx->side[0] && ((lg ? 1 : 0) + (mg ? 1 : 0) + ((ug || hg) ? 1 : 0)) >= 2;
    if (fork) {
        DT_HIP(hipEventRecord(ctx->ev_fork, s));
        if (lg) {
            DT_HIP(hipStreamWaitEvent(ctx->side[0], ctx->ev_fork, 0));
            sl = ctx->side[0];
        }
        if (mg) {
            DT_HIP(hipStreamWaitEvent(ctx->side[1], ctx->ev_fork, 0));
            sm = ctx->side[1];
        }
    }
    if (lg) {
        prof_begin(ctx, kProfLight, sl);
        if (cells)
            k_light<true, kLightBlock><<<lg, kLightBlock, 0, sl>>>(p.lr, p.light,
                g->eoff.as<uint32_t>(), g->key.as<uint64_t>(), q, part, cells_dev);
        else
            k_light<false, kLightBlock><<<lg, kLightBlock, 0, sl>>>(p.lr, p.light,
                g->eoff.as<uint32_t>(), g->key.as<uint64_t>(), q, part, nullptr);
        prof_end(ctx, kProfLight, sl);
        DT_HIP(hipGetLastError());
    }
    if (mg) {
        prof_begin(ctx, kProfMedium, sm);
        if (cells)
            k_medium<true, 256><<<mg, 256, 0, sm>>>(p.mr, p.medium, p.mitems,
                g->eoff.as<uint32_t>(),
                g->key.as<uint64_t>(), q, part + 8 * ((uint64_t)lg + hg), cells_dev);
        else
            k_medium<false, 256><<<mg, 256, 0, sm>>>(p.mr, p.medium, p.mitems,
                g->eoff.as<uint32_t>(),
                g->key.as<uint64_t>(), q, part + 8 * ((uint64_t)lg + hg), nullptr);
        prof_end(ctx, kProfMedium, sm);
        DT_HIP(hipGetLastError());
    }
    if (ug) {
        const UQuery u = unit_query(q);
        int64_t *up = part + 8 * ((uint64_t)lg + hg + mg);
        prof_begin(ctx, kProfUnit, s);
        if (cells)
            k_unit<true, kUnitBlock><<<ug, kUnitBlock, 0, s>>>(p.ub, p.ue, S.unit.as<uint4>(), u, up, cells_dev);
        else
            k_unit<false, kUnitBlock><<<ug, kUnitBlock, 0, s>>>(p.ub, p.ue, S.unit.as<uint4>(), u, up, nullptr);
        prof_end(ctx, kProfUnit, s);
        DT_HIP(hipGetLastError());
    }
    if (p.heavy_bytes) {
        int64_t *P = reinterpret_cast<int64_t *>(sv.heavy);
        uint32_t *clip = reinterpret_cast<uint32_t *>(P + S.n_slots * kVals);
        k_heavy_clip<<<grid_for(S.n_heavy, 256), 256, 0, s>>>(S.n_heavy, S.heavy.as<uint32_t>(),
            g->eoff.as<uint32_t>(), g->key.as<uint64_t>(), q, clip);
        DT_HIP(hipGetLastError());
        prof_begin(ctx, kProfHeavyPrefix, s);
        k_heavy_prefix<<<(unsigned)(4 * S.n_heavy), kPrefixBlock, 0, s>>>(S.n_heavy, S.heavy.as<uint32_t>(),
            g->eoff.as<uint32_t>(), g->key.as<uint64_t>(), clip, S.hslot.as<uint64_t>(), S.n_slots, q, P);
        prof_end(ctx, kProfHeavyPrefix, s);
        DT_HIP(hipGetLastError());
        const unsigned cb = g->tuning.heavy_chunk;
        prof_begin(ctx, kProfHeavyCount, s);
        if (cells) {
            if (cb == 256)
                k_heavy_count<true, 256><<<hg, 256, 0, s>>>(S.n_chunks, S.chunks.as<uint32_t>(),
                    S.heavy.as<uint32_t>(), g->eoff.as<uint32_t>(), g->key.as<uint64_t>(), clip,
                    S.hslot.as<uint64_t>(), S.n_slots, P, q, part + 8 * (uint64_t)lg, cells_dev);
            else
                return fail(DT_EINVAL, "heavy_chunk %u not compiled", cb);
        } else {
            if (cb == 256)
                k_heavy_count<false, 256><<<hg, 256, 0, s>>>(S.n_chunks, S.chunks.as<uint32_t>(),
                    S.heavy.as<uint32_t>(), g->eoff.as<uint32_t>(), g->key.as<uint64_t>(), clip,
                    S.hslot.as<uint64_t>(), S.n_slots, P, q, part + 8 * (uint64_t)lg, nullptr);
            else
                return fail(DT_EINVAL, "heavy_chunk %u not compiled", cb);
        }
        prof_end(ctx, kProfHeavyCount, s);
        DT_HIP(hipGetLastError());
    }
    if (fork) {
        if (lg) {
            DT_HIP(hipEventRecord(ctx->ev_join[0], sl));
            DT_HIP(hipStreamWaitEvent(s, ctx->ev_join[0], 0));
        }
        if (mg) {
            DT_HIP(hipEventRecord(ctx->ev_join[1], sm));
            DT_HIP(hipStreamWaitEvent(s, ctx->ev_join[1], 0));
        }
    }
    if (!cells) {
        prof_begin(ctx, kProfReduce, s);
        k_reduce<<<1, 256, 0, s>>>(n_part, part, out8_dev);
        prof_end(ctx, kProfReduce, s);
        DT_HIP(hipGetLastError());
    }
    return DT_OK;
}

// Plan one count, grow the scratch sc to its needs, and enqueue it on stream s.
int count_enqueue(dt_graph *g, const DQuery &q, int64_t *out8_dev, hipStream_t s, bool cells,
                  int64_t *cells_dev, Scratch &sc, unsigned parts) {
    CountPlan p;
    count_plan(g, q, parts, p);
    DT_TRY(ensure(g->ctx, sc.partials, p.part_bytes));
    if (p.heavy_bytes) DT_TRY(ensure(g->ctx, sc.heavy_vals, p.heavy_bytes));
    ScratchView sv;
    sv.part = sc.partials.as<int64_t>();
    sv.part_bytes = sc.partials.bytes;
    sv.heavy = sc.heavy_vals.as<uint8_t>();
    sv.heavy_bytes = p.heavy_bytes ? sc.heavy_vals.bytes : 0;
    return count_launch(g, q, p, out8_dev, s, cells, cells_dev, sv);
}

void count_reduce(uint64_t n_part, const int64_t *part, int64_t *out8_dev, hipStream_t s) {
    k_reduce<<<1, 256, 0, s>>>(n_part, part, out8_dev);
}

// A sweep: k <= kSweepMax queries with one window.  The unit, light and medium kernels visit each
// triangle's data once per pass and count it for every delta triple: records and lists are read
// once, the light path enumerates each triangle's pairs once, the medium path finds each entry's
// close pairs once (for the largest d13); only the delta-dependent searches repeat.  The rare heavy
// triangles are counted per query first, and the reduction adds the rest to those sums.
int count_sweep_enqueue(dt_graph *g, const DQuery *qs, uint32_t k, int64_t *out_dev, hipStream_t s, Scratch &sc) {
    dt_ctx *ctx = g->ctx;
    Schedule &S = g->sched;
    if (k == 0 || k > kSweepMax) return fail(DT_EINVAL, "a sweep pass takes 1..%u queries", kSweepMax);
    SweepQ Q{};
    Q.k = k;
    Q.d13max = 0;
    for (uint32_t j = 0; j < k; ++j) {
        Q.q[j] = qs[j];
        Q.u[j] = unit_query(qs[j]);
        Q.d13max = qs[j].d13 > Q.d13max ? qs[j].d13 : Q.d13max;
    }
    const DQuery &q0 = qs[0];   // the window (and so every range) is the same for all k
    // heavy triangles: one count per query, written to out_dev
    const bool heavy = S.n_chunks > 0;
    if (heavy)
        for (uint32_t j = 0; j < k; ++j) DT_TRY(count_enqueue(g, qs[j], out_dev + 8 * j, s, false, nullptr, sc, 4));
    Ranges lr, mr;
    cell_ranges(S.light_cells, S.cell_shift, q0, lr);
    cell_ranges(S.mitem_cells, S.cell_shift, q0, mr);
    const uint64_t nl = lr.pre[lr.n], nmi = mr.pre[mr.n];
    const uint32_t *light = (q0.windowed ? S.light_w : S.light).as<uint32_t>();
    const uint32_t *medium = (q0.windowed ? S.medium_w : S.medium).as<uint32_t>();
    const uint32_t *mitems = (q0.windowed ? S.mitems_w : S.mitems).as<uint32_t>();
    const unsigned lg = nl ? (unsigned)std::min<uint64_t>((nl + kLightBlock - 1) / kLightBlock, (uint64_t)ctx->num_cus * 16) : 0;
    const unsigned lgx = lg ? ((lg + 7) / 8) * 8 : 0;
    const unsigned mg = nmi ? (unsigned)std::min<uint64_t>((nmi + 255) / 256, (uint64_t)ctx->num_cus * 8) : 0;
    uint64_t ub = 0, ue = 0;
    if (S.n_unit) unit_range(g, q0, &ub, &ue);
    const unsigned ug = ue > ub ? (unsigned)std::min<uint64_t>((ue - ub + kUnitPerBlock - 1) / kUnitPerBlock,
                                                               (uint64_t)ctx->num_cus * 8) : 0;
    const uint64_t n_slot = (uint64_t)ug + lgx + mg;
    DT_TRY(ensure(ctx, sc.sweep_partials, (n_slot + 1) * k * 8 * sizeof(int64_t)));
    int64_t *part = sc.sweep_partials.as<int64_t>();
    // the light and medium passes run on the side streams, beside the unit pass (as in a count)
    hipStream_t sl = s, sm = s;
    const bool fork = ctx->side[0] && ((ug ? 1 : 0) + (lgx ? 1 : 0) + (mg ? 1 : 0)) >= 2;
    if (fork) {
        DT_HIP(hipEventRecord(ctx->ev_fork, s));
        if (lgx) {
            DT_HIP(hipStreamWaitEvent(ctx->side[0], ctx->ev_fork, 0));
            sl = ctx->side[0];
        }
        if (mg) {
            DT_HIP(hipStreamWaitEvent(ctx->side[1], ctx->ev_fork, 0));
            sm = ctx->side[1];
        }
    }
    if (ug) {
        prof_begin(ctx, kProfUnit, s);
        k_unit_sweep<kUnitBlock><<<ug, kUnitBlock, 0, s>>>(ub, ue, S.unit.as<uint4>(), Q, part, 0);
        prof_end(ctx, kProfUnit, s);
        DT_HIP(hipGetLastError());
    }
    if (lgx) {
        prof_begin(ctx, kProfLight, sl);
        k_light_sweep<kLightBlock><<<lgx, kLightBlock, 0, sl>>>(lr, light, g->eoff.as<uint32_t>(), g->key.as<uint64_t>(),
                                                                Q, part, ug);
        prof_end(ctx, kProfLight, sl);
        DT_HIP(hipGetLastError());
    }
    if (mg) {
        prof_begin(ctx, kProfMedium, sm);
        k_medium_sweep<256><<<mg, 256, 0, sm>>>(mr, medium, mitems, g->eoff.as<uint32_t>(), g->key.as<uint64_t>(),
                                                Q, part, (uint64_t)ug + lgx);
        prof_end(ctx, kProfMedium, sm);
        DT_HIP(hipGetLastError());
    }
    if (fork) {
        if (lgx) {
            DT_HIP(hipEventRecord(ctx->ev_join[0], sl));
            DT_HIP(hipStreamWaitEvent(s, ctx->ev_join[0], 0));
        }
        if (mg) {
            DT_HIP(hipEventRecord(ctx->ev_join[1], sm));
            DT_HIP(hipStreamWaitEvent(s, ctx->ev_join[1], 0));
        }
    }
    prof_begin(ctx, kProfReduce, s);
    k_reduce_sweep<<<k, 256, 0, s>>>(n_slot, k, part, out_dev, heavy ? 1 : 0);
    prof_end(ctx, kProfReduce, s);
    DT_HIP(hipGetLastError());
    return DT_OK;
}

}  // namespace dt
