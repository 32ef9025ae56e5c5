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
#include <type_traits>

#include "count_dev.h"

namespace dt {

using namespace cdev;

namespace {

// ACC: Acc<false> (int64 type counts), Acc<true> (the 48 cells by atomics, no partials) or AccW
// (128-bit type counts, 16-word partial slots)
template <class ACC> constexpr bool kCells = std::is_same<ACC, Acc<true>>::value;

template <class ACC, unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_light(Ranges R, const uint32_t *__restrict__ tri, const uint32_t *__restrict__ eoff,
        const uint64_t *__restrict__ key, DQuery q, int64_t *__restrict__ partial,
        int64_t *__restrict__ cells, unsigned long long *__restrict__ visits) {
    ACC acc;
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
    add_visits(visits, acc.visits);
    if (!kCells<ACC>) acc_store<BLOCK>(acc, partial, blockIdx.x);
}

// medium path: wave w takes the 64 entries from 64 w on, then those from 64 (w + W) on, ...;
// with lev (windowed copies) entries of triangles below the query's level are skipped
template <class ACC, unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_medium(Ranges R, const uint32_t *__restrict__ med, const uint32_t *__restrict__ ent,
         const uint8_t *__restrict__ lev, const uint32_t *__restrict__ eoff, const uint64_t *__restrict__ key,
         DQuery q, int64_t *__restrict__ partial, int64_t *__restrict__ cells, unsigned long long *__restrict__ visits) {
    ACC acc;
    acc.cells = cells;
    const unsigned lane = threadIdx.x & 63;
    const uint64_t n_ent = R.pre[R.n];
    const uint64_t W = (uint64_t)gridDim.x * (BLOCK / 64);
    uint32_t r = 0;
    uint64_t vis = 0;
    for (uint64_t b = ((uint64_t)blockIdx.x * (BLOCK / 64) + threadIdx.x / 64) * 64; b < n_ent; b += W * 64) {
        const uint64_t j = b + lane;
        const bool active = j < n_ent;
        // one visit per outer edge, plus the wavefront's close pairs (counted by lane 0)
        const uint32_t pairs = medium_lanes(med, ent, active ? range_at(R, r, j) : 0, active, eoff, key, q, acc, lane, lev);
        vis += (active ? 1u : 0u) + (lane == 0 ? pairs : 0u);
    }
    add_visits(visits, vis);
    if (!kCells<ACC>) acc_store<BLOCK>(acc, partial, blockIdx.x);
}

// unit path: block b takes a contiguous run of the records [beg, end)
template <class ACC, unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_unit(uint64_t beg, uint64_t end, const uint4 *__restrict__ rec, UQuery u, int64_t *__restrict__ partial,
       int64_t *__restrict__ cells, unsigned long long *__restrict__ visits) {
    constexpr bool CELLS = kCells<ACC>;
    const uint64_t n = end - beg;
    const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b = beg + (uint64_t)blockIdx.x * per;
    const uint64_t e = b + per < end ? b + per : end;
    uint32_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (b < e) unit_run<CELLS, BLOCK>(rec, b, e, u, c, cells);
    if (visits && threadIdx.x == 0 && e > b) atomicAdd(visits, (unsigned long long)(e - b));
    if (!CELLS) {
        ACC acc;
#pragma unroll
        for (int j = 0; j < 8; ++j) acc.t[j] = c[j];
        acc_store<BLOCK>(acc, partial, blockIdx.x);
    }
}

// ---------------------------------------------------------------------------------------------
// heavy path (the per-item bodies are in count_dev.h, shared with the batched kernel)
// ---------------------------------------------------------------------------------------------
// window-clipped bounds of the six lists of every heavy triangle of the query
__global__ void k_heavy_clip(HeavyArgs A, uint64_t n_q) {
    const uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h < n_q) heavy_clip_one(A, h);
}

// phase 1 of the prefix pass over prefix chunks [A.pb, pe)
__global__ void __launch_bounds__(kPrefixBlock)
k_heavy_prefix_local(HeavyArgs A, uint64_t pe, unsigned long long *__restrict__ visits) {
    uint64_t vis = 0;
    for (uint64_t c = A.pb + blockIdx.x; c < pe; c += gridDim.x) heavy_prefix_local_chunk(A, c, vis);
    add_visits(visits, vis);
}

// phase 2: the carries between the chunks of each list (a thread per chunk, the list's first works)
__global__ void k_heavy_prefix_scan(HeavyArgs A, uint64_t pe) {
    const uint64_t c = A.pb + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < pe) heavy_prefix_scan_list(A, c, pe);
}

// phase 3: every chunk adds its carry
__global__ void __launch_bounds__(kPrefixBlock)
k_heavy_prefix_add(HeavyArgs A, uint64_t pe) {
    for (uint64_t c = A.pb + blockIdx.x; c < pe; c += gridDim.x) heavy_prefix_add_chunk(A, c);
}

// the count pass: chunks [cb, ce) of 256 source edges (of the four lists in a row) each
template <class ACC, unsigned BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_heavy_count(HeavyArgs A, uint64_t cb, uint64_t ce, int64_t *__restrict__ partial, int64_t *__restrict__ cells,
              unsigned long long *__restrict__ visits) {
    ACC acc;
    acc.cells = cells;
    for (uint64_t ch = cb + blockIdx.x; ch < ce; ch += gridDim.x) heavy_count_chunk(A, ch, acc);
    add_visits(visits, acc.visits);
    if (!kCells<ACC>) acc_store<BLOCK>(acc, partial, blockIdx.x);
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

// the 128-bit form: 16-word partials into 16 words (low, high per type)
__global__ void __launch_bounds__(256)
k_reduce_w(uint64_t n_part, const int64_t *__restrict__ partial, int64_t *__restrict__ out16) {
    AccW acc;
    for (uint64_t i = threadIdx.x; i < n_part; i += 256) {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            acc.t[j] += ((unsigned __int128)(uint64_t)partial[16 * i + 2 * j + 1] << 64) | (uint64_t)partial[16 * i + 2 * j];
    }
    block_store_w<256>(acc.t, out16);
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
    uint32_t qlev;    // its level: the pass's medium / heavy split
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
               const uint8_t *__restrict__ lev, const uint32_t *__restrict__ eoff, const uint64_t *__restrict__ key, SweepQ Q,
               int64_t *__restrict__ part, uint64_t slot0) {
    __shared__ unsigned long long s_sw[BLOCK / 64][kSweepMax * 8];
    for (unsigned x = threadIdx.x; x < (BLOCK / 64) * kSweepMax * 8; x += BLOCK) (&s_sw[0][0])[x] = 0;
    __syncthreads();
    unsigned long long *sw = s_sw[threadIdx.x / 64];
    const unsigned lane = threadIdx.x & 63;
    const uint64_t n_ent = R.pre[R.n];
    const uint64_t W = (uint64_t)gridDim.x * (BLOCK / 64);
    DQuery qr = Q.q[0];   // the window, the widest closeness and the pass's medium / heavy split
    qr.d13 = Q.d13max;
    qr.qlev = Q.qlev;
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
                          lane, lev);
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
    q.qlev = query_level(d13);
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

void medium_ranges(const dt_graph *g, const DQuery &q, Ranges &r, const uint8_t **lev) {
    const Schedule &S = g->sched;
    if (q.windowed) {
        cell_ranges(S.mitem_cells, S.cell_shift, q, r);
        *lev = S.mlev_w.as<uint8_t>();
        return;
    }
    // whole span: the entries of the always-medium triangles and of the contested ones at or above
    // the query's level, a prefix of the list
    const uint64_t e = S.med_item_at[q.qlev < kLevels ? q.qlev : kLevels];
    r.n = e ? 1 : 0;
    r.pre[0] = 0;
    if (e) {
        r.b[0] = 0;
        r.pre[1] = e;
    }
    *lev = nullptr;
}

void heavy_range(const dt_graph *g, const DQuery &q, HeavyRange &h) {
    const Schedule &S = g->sched;
    const uint32_t l = q.qlev < kLevels ? q.qlev : kLevels;
    h.hb = S.heavy_tri_at[l];
    h.cb = S.heavy_chunk_at[l];
    h.pb = S.heavy_pchunk_at[l];
    h.slot_base = S.heavy_slot_at[l];
    h.n = S.n_heavy - h.hb;
    h.scratch_bytes = h.n ? (S.n_slots - h.slot_base) * kVals * sizeof(int64_t) + 12 * 4 * h.n +
                                (S.n_pchunks - h.pb) * kVals * sizeof(int64_t) + 512
                          : 0;
}

void heavy_args(const dt_graph *g, const DQuery &q, const HeavyRange &hr, uint8_t *scratch, HeavyArgs &A) {
    const Schedule &S = g->sched;
    const uint64_t ns = S.n_slots - hr.slot_base, npc = S.n_pchunks - hr.pb;
    A.heavy = S.heavy.as<uint32_t>();
    A.pchunks = S.pchunks.as<uint32_t>();
    A.chunks = S.chunks.as<uint32_t>();
    A.eoff = g->eoff.as<uint32_t>();
    A.key = g->key.as<uint64_t>();
    A.hslot = S.hslot.as<uint64_t>();
    A.hb = hr.hb;
    A.pb = hr.pb;
    A.slot_base = hr.slot_base;
    A.ns = ns;
    A.P = reinterpret_cast<int64_t *>(scratch);
    A.T = A.P + ns * kVals;
    A.clip = reinterpret_cast<uint32_t *>(A.T + npc * kVals);
    A.q = q;
}

void count_plan(const dt_graph *g, const DQuery &q, unsigned parts, CountPlan &p) {
    const dt_ctx *ctx = g->ctx;
    const Schedule &S = g->sched;
    p.parts = parts;
    const bool do_light = parts & 1, do_medium = parts & 2, do_heavy = parts & 4;
    // the parts of the light and medium lists the query sees (window cells; the medium / heavy
    // split of its level)
    cell_ranges(S.light_cells, S.cell_shift, q, p.lr);
    medium_ranges(g, q, p.mr, &p.mlev);
    const uint64_t nl = p.lr.pre[p.lr.n], nmi = p.mr.pre[p.mr.n];
    p.light = (q.windowed ? S.light_w : S.light).as<uint32_t>();
    p.medium = (q.windowed ? S.medium_w : S.medium).as<uint32_t>();
    p.mitems = (q.windowed ? S.mitems_w : S.mitems).as<uint32_t>();
    const CountGeom &G = g->geom;
    const unsigned light_grid = (nl && do_light) ? (unsigned)std::min<uint64_t>(
        (nl + kLightBlock - 1) / kLightBlock, (uint64_t)ctx->num_cus * G.light_bpc) : 0;
    p.lg = light_grid ? ((light_grid + 7) / 8) * 8 : 0;
    heavy_range(g, q, p.hr);
    if (!do_heavy) p.hr.n = 0;
    p.hg = p.hr.n ? (unsigned)std::min<uint64_t>(S.n_chunks - p.hr.cb, (uint64_t)ctx->num_cus * 16) : 0;
    p.mg = (nmi && do_medium) ? (unsigned)std::min<uint64_t>((nmi + 255) / 256, (uint64_t)ctx->num_cus * G.medium_bpc) : 0;
    p.ub = p.ue = 0;
    if (S.n_unit && (parts & 8)) unit_range(g, q, &p.ub, &p.ue);
    p.ug = p.ue > p.ub ? (unsigned)std::min<uint64_t>((p.ue - p.ub + kUnitPerBlock - 1) / kUnitPerBlock,
                                                      (uint64_t)ctx->num_cus * 8) : 0;
    p.n_part = (uint64_t)p.lg + p.hg + p.mg + p.ug;
    // graphs whose counts may pass 2^63 are counted in 128 bits (16-word partials, 16-word result)
    p.wide = (g->sum_sigma3 >> 63) != 0;
    p.part_bytes = (p.n_part + 1) * (p.wide ? 16 : 8) * sizeof(int64_t);
    p.heavy_bytes = p.hr.n ? p.hr.scratch_bytes : 0;
}

// The four paths' kernels of a planned count with accumulator ACC: the light and heavy ones on sl,
// the medium one on sm, the unit one on s; partial slots of 8 words (16 for AccW) in the order
// light, heavy, medium, unit.
template <class ACC>
int launch_paths(dt_graph *g, const DQuery &q, const CountPlan &p, const ScratchView &sv, hipStream_t s,
                 hipStream_t sl, hipStream_t sm, int64_t *cells_dev, unsigned long long *visits) {
    dt_ctx *ctx = g->ctx;
    Schedule &S = g->sched;
    constexpr uint64_t W = std::is_same<ACC, AccW>::value ? 16 : 8;
    const unsigned lg = p.lg, hg = p.hg, mg = p.mg, ug = p.ug;
    int64_t *part = sv.part;
    const uint32_t *eoff = g->eoff.as<uint32_t>();
    const uint64_t *key = g->key.as<uint64_t>();
    if (lg) {
        prof_begin(ctx, kProfLight, sl);
        k_light<ACC, kLightBlock><<<lg, kLightBlock, 0, sl>>>(p.lr, p.light, eoff, key, q, part, cells_dev, visits);
        prof_end(ctx, kProfLight, sl);
        DT_HIP(hipGetLastError());
    }
    if (mg) {
        int64_t *mp = part + W * ((uint64_t)lg + hg);
        prof_begin(ctx, kProfMedium, sm);
        k_medium<ACC, 256><<<mg, 256, 0, sm>>>(p.mr, p.medium, p.mitems, p.mlev, eoff, key, q, mp, cells_dev, visits);
        prof_end(ctx, kProfMedium, sm);
        DT_HIP(hipGetLastError());
    }
    if (ug) {
        const UQuery u = unit_query(q);
        int64_t *up = part + W * ((uint64_t)lg + hg + mg);
        prof_begin(ctx, kProfUnit, s);
        k_unit<ACC, kUnitBlock><<<ug, kUnitBlock, 0, s>>>(p.ub, p.ue, S.unit.as<uint4>(), u, up, cells_dev, visits);
        prof_end(ctx, kProfUnit, s);
        DT_HIP(hipGetLastError());
    }
    if (p.hr.n) {
        const HeavyRange &hr = p.hr;
        const uint64_t npc = S.n_pchunks - hr.pb;
        HeavyArgs A;
        heavy_args(g, q, hr, sv.heavy, A);
        k_heavy_clip<<<grid_for(hr.n, 256), 256, 0, sl>>>(A, hr.n);
        DT_HIP(hipGetLastError());
        const unsigned pgrid = (unsigned)std::min<uint64_t>(npc, (uint64_t)ctx->num_cus * 16);
        prof_begin(ctx, kProfHeavyPrefix, sl);
        k_heavy_prefix_local<<<pgrid, kPrefixBlock, 0, sl>>>(A, S.n_pchunks, visits);
        DT_HIP(hipGetLastError());
        k_heavy_prefix_scan<<<grid_for(npc, 256), 256, 0, sl>>>(A, S.n_pchunks);
        DT_HIP(hipGetLastError());
        k_heavy_prefix_add<<<pgrid, kPrefixBlock, 0, sl>>>(A, S.n_pchunks);
        prof_end(ctx, kProfHeavyPrefix, sl);
        DT_HIP(hipGetLastError());
        const unsigned cb = g->tuning.heavy_chunk;
        if (cb != 256) return fail(DT_EINVAL, "heavy_chunk %u not compiled", cb);
        int64_t *hp = part + W * (uint64_t)lg;
        prof_begin(ctx, kProfHeavyCount, sl);
        k_heavy_count<ACC, 256><<<hg, 256, 0, sl>>>(A, hr.cb, S.n_chunks, hp, cells_dev, visits);
        prof_end(ctx, kProfHeavyCount, sl);
        DT_HIP(hipGetLastError());
    }
    return DT_OK;
}

// Enqueue one planned count on stream s: partials -> out8_dev (int64[8]); cells mode accumulates the
// 48 cells into cells_dev (zeroed here) instead.  The scratch must hold the plan's needs.  With
// visits, the kernels add the pairs and list elements they iterate over to *visits.
int count_launch(dt_graph *g, const DQuery &q, const CountPlan &p, int64_t *out8_dev, hipStream_t s, bool cells,
                 int64_t *cells_dev, const ScratchView &sv, unsigned long long *visits) {
    dt_ctx *ctx = g->ctx;
    prof_clear(ctx, false);
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
    // The paths are independent (each writes its own partial slots): when more than one has work,
    // the light and then the heavy kernels run on the context's first side stream and the medium
    // kernel on the second, forked from s here and joined back before the reduction, beside the
    // unit kernel on s, so that their latency-bound tails overlap.
    hipStream_t sl = s, sm = s;
    const bool fork = ctx->side[0] && ((lg || hg ? 1 : 0) + (mg ? 1 : 0) + (ug ? 1 : 0)) >= 2;
    if (fork) {
        DT_HIP(hipEventRecord(ctx->ev_fork, s));
        if (lg || hg) {
            DT_HIP(hipStreamWaitEvent(ctx->side[0], ctx->ev_fork, 0));
            sl = ctx->side[0];
        }
        if (mg) {
            DT_HIP(hipStreamWaitEvent(ctx->side[1], ctx->ev_fork, 0));
            sm = ctx->side[1];
        }
    }
    if (cells) {
        DT_TRY(launch_paths<Acc<true>>(g, q, p, sv, s, sl, sm, cells_dev, visits));
    } else if (p.wide) {
        DT_TRY(launch_paths<AccW>(g, q, p, sv, s, sl, sm, nullptr, visits));
    } else {
        DT_TRY(launch_paths<Acc<false>>(g, q, p, sv, s, sl, sm, nullptr, visits));
    }
    if (fork) {
        if (lg || hg) {
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
        if (p.wide) k_reduce_w<<<1, 256, 0, s>>>(n_part, part, out8_dev);
        else k_reduce<<<1, 256, 0, s>>>(n_part, part, out8_dev);
        prof_end(ctx, kProfReduce, s);
        DT_HIP(hipGetLastError());
    }
    return DT_OK;
}

// Plan one count, grow the scratch sc to its needs, and enqueue it on stream s.
int count_enqueue(dt_graph *g, const DQuery &q, int64_t *out8_dev, hipStream_t s, bool cells,
                  int64_t *cells_dev, Scratch &sc, unsigned parts, unsigned long long *visits) {
    CountPlan p;
    count_plan(g, q, parts, p);
    DT_TRY(ensure(g->ctx, sc.partials, p.part_bytes));
    if (p.heavy_bytes) DT_TRY(ensure(g->ctx, sc.heavy_vals, p.heavy_bytes));
    ScratchView sv;
    sv.part = sc.partials.as<int64_t>();
    sv.part_bytes = sc.partials.bytes;
    sv.heavy = sc.heavy_vals.as<uint8_t>();
    sv.heavy_bytes = p.heavy_bytes ? sc.heavy_vals.bytes : 0;
    return count_launch(g, q, p, out8_dev, s, cells, cells_dev, sv, visits);
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
    // one medium / heavy split for the whole pass: the level of the largest d13 (the medium pass
    // finds close pairs at that distance for every triple)
    uint32_t qlm = 0;
    for (uint32_t j = 0; j < k; ++j) qlm = qs[j].qlev > qlm ? qs[j].qlev : qlm;
    // heavy triangles: one count per query, written to out_dev
    DQuery qh = q0;
    qh.qlev = qlm;
    HeavyRange hr;
    heavy_range(g, qh, hr);
    const bool heavy = hr.n > 0;
    if (heavy)
        for (uint32_t j = 0; j < k; ++j) {
            DQuery qq = qs[j];
            qq.qlev = qlm;
            DT_TRY(count_enqueue(g, qq, out_dev + 8 * j, s, false, nullptr, sc, 4));
        }
    Q.qlev = qlm;
    Ranges lr, mr;
    const uint8_t *mlev = nullptr;
    cell_ranges(S.light_cells, S.cell_shift, q0, lr);
    medium_ranges(g, qh, mr, &mlev);
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
        k_medium_sweep<256><<<mg, 256, 0, sm>>>(mr, medium, mitems, mlev, g->eoff.as<uint32_t>(), g->key.as<uint64_t>(),
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
