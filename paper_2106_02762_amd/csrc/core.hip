// Degeneracy ordering from core numbers (Section 3 orders the vertices so that each has at most
// degeneracy-many neighbours after it; the degeneracy is the largest core number).  The library's
// second way to order a graph (order_method 1); the level-by-level peel in peel.hip is the default.
// On the power-law graphs measured here this one needs far fewer grid-wide steps (about 40 h-index
// phases and 30 removal rounds against hundreds of levels) but reads the rows of high-degree
// vertices again in most phases, and random gathers of neighbour bounds, not synchronisation, set
// its time: about 3x the level peel's on a 61M-edge graph.
//
// Two stages on one cooperative grid, separated by grid barriers instead of launches:
//
// 1. Core numbers by h-index iteration.  Every vertex holds an upper bound h(v) on its core
//    number, first its degree.  Processing v replaces h(v) by the h-index of its neighbours'
//    bounds capped at h(v): the largest k <= h(v) such that at least k neighbours have a bound
//    >= k.  While every bound is >= its vertex's core number this value is too (v has core(v)
//    neighbours in the core(v)-core, each with a bound >= core(v)), so bounds stay bounds and
//    only fall.  Once no bound changes, the vertices of bound >= k induce a subgraph of minimum
//    degree >= k for every k, so every bound is also <= the core number: the bounds are the core
//    numbers.  Lowering h(u) can only lower the h-index of a neighbour whose bound is above the
//    new h(u), so only those are processed again, in the next phase; a bound read while another
//    block lowers it is still a bound, and the lowering schedules the reader again.
// 2. The ordering, by peeling every shell (the vertices of one core number c) at once.  d(v)
//    counts the neighbours of core >= core(v).  A vertex of the c-shell is removed once d(v) <= c,
//    which lowers d of its shell neighbours not yet removed; in the c-core, repeatedly removing
//    vertices of degree <= c removes exactly the c-shell, so every vertex is removed.  The
//    ordering sorts by (core, round of removal); vertices of one round may come in any order.
//    When v is removed, each neighbour placed after it -- of higher core, or of v's shell and
//    removed in the same or a later round -- is counted in d(v) <= core(v): the out-degree bound
//    Theorem 1 rests on.
//
// Work is spread by degree: a vertex whose row has at most kLaneDeg entries takes one lane, one of
// up to kWaveDeg entries a wavefront, a longer one the whole workgroup; each kind has its own region
// of the work lists, whose entries are taken through per-phase counters, and a vertex is listed at
// most once per phase.  A wavefront's or workgroup's vertex gets its h-index from a histogram of its
// neighbours' bounds in LDS: one pass when h(v) fits the histogram, otherwise a pass with buckets of
// several values and then one over the bucket that holds the answer.  A lane's vertex gets it by
// binary search over counts.  Both stages need a number of phases that grows with the longest
// chain of dependent changes (tens on power-law graphs; a path of p vertices needs about p/2).
#include "internal.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 1024;
constexpr unsigned kWaves = kBlock / 64;
constexpr uint32_t kLaneDeg = 32;      // rows of at most this many entries: one lane per vertex
constexpr uint32_t kWaveDeg = 4096;    // rows of at most this many entries: one wavefront
constexpr uint32_t kWaveHist = 1024;   // histogram words of one wavefront
constexpr uint32_t kBlockHist = kWaves * kWaveHist;   // the same LDS words, for the workgroup
constexpr uint32_t kUnset = 0xffffffffu;
constexpr long kSpinLimit = 1l << 26;

enum Stage { kHindex = 0, kDegree = 1, kRemove = 2 };

struct CoreCtl {
    unsigned arrived;        // barrier arrivals (only ever increases)
    unsigned error;          // 1 barrier timeout, 2 list overflow, 4 and 16 checks, 8 phase limit
    unsigned flag[3];        // per phase mod 3: the phase scheduled work for the next one
    unsigned iters;          // phases of the h-index stage
    unsigned rounds;         // removal rounds
    unsigned kappa;          // largest core number
};

__device__ __forceinline__ unsigned ld_relaxed(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier: arrivals only ever increase, and every block passes the same barriers, so a
// barrier is complete once target (gridDim.x times the barriers so far) arrivals are counted.  One
// that waits far longer than the whole computation could take sets an error flag and lets its
// block go.
__device__ void grid_barrier(CoreCtl *ctl, unsigned &target) {
    target += gridDim.x;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned a = atomicAdd(&ctl->arrived, 1u) + 1;
        if (a < target) {
            long spins = 0;
            while (__hip_atomic_load(&ctl->arrived, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kSpinLimit) {
                    atomicOr(&ctl->error, 1u);
                    break;
                }
            }
        } else {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t row_class(uint32_t len) {
    return len <= kLaneDeg ? 0u : (len <= kWaveDeg ? 1u : 2u);
}

__device__ __forceinline__ unsigned wave_sum(unsigned x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// sum of x over the lanes above this one
__device__ __forceinline__ unsigned wave_suffix_excl(unsigned x, unsigned lane) {
    unsigned incl = x;   // inclusive prefix from lane 0
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(incl, o, 64);
        if (lane >= (unsigned)o) incl += y;
    }
    return __shfl(incl, 63, 64) - incl;
}

// ordering of LDS accesses among the lanes of one wavefront (its LDS operations complete in order;
// this keeps the compiler from moving them across)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// A group is one wavefront (G = 64) or the workgroup (G = kBlock); gl is the thread's index in it.
template <unsigned G>
__device__ __forceinline__ void grp_sync() {
    if constexpr (G == 64) wave_sync();
    else __syncthreads();
}

template <unsigned G>
__device__ __forceinline__ unsigned grp_sum(unsigned x, unsigned *s_red) {
    x = wave_sum(x);
    if constexpr (G == 64) {
        return x;
    } else {
        const unsigned wave = threadIdx.x / 64;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) s_red[wave] = x;
        __syncthreads();
        unsigned t = 0;
#pragma unroll
        for (unsigned w = 0; w < kWaves; ++w) t += s_red[w];
        return t;
    }
}

template <unsigned G>
__device__ __forceinline__ unsigned grp_suffix_excl(unsigned x, unsigned *s_red) {
    const unsigned lane = threadIdx.x & 63;
    const unsigned in_wave = wave_suffix_excl(x, lane);
    if constexpr (G == 64) {
        return in_wave;
    } else {
        const unsigned wave = threadIdx.x / 64;
        const unsigned tot = wave_sum(x);
        __syncthreads();
        if (lane == 0) s_red[wave] = tot;
        __syncthreads();
        unsigned above = 0;
        for (unsigned w = wave + 1; w < kWaves; ++w) above += s_red[w];
        return in_wave + above;
    }
}

// Number of bucket indices i in [0, nb) with  above + sum_{i' >= i} hist[i'] >= lo + i * B
// (true for a prefix of the indices: the left side falls and the right side grows with i).
template <unsigned G>
__device__ unsigned grp_prefix_true(const uint32_t *hist, uint32_t nb, uint32_t above, uint32_t lo, uint32_t B,
                                    unsigned gl, unsigned *s_red) {
    const uint32_t q = (nb + G - 1) / G;
    const uint32_t s = min(gl * q, nb), e = min(s + q, nb);
    unsigned local = 0;
    for (uint32_t i = s; i < e; ++i) local += hist[i];
    uint64_t acc = (uint64_t)above + grp_suffix_excl<G>(local, s_red);
    unsigned cnt = 0;
    for (uint32_t i = e; i-- > s;) {
        acc += hist[i];
        cnt += acc >= (uint64_t)lo + (uint64_t)i * B;
    }
    return grp_sum<G>(cnt, s_red);
}

// h-index of the vertex with row [b, e) and bound hv (> 0), capped at hv, by the group.  The
// window [lo, top] holds the answer and `above` counts the bounds beyond it; a pass counts the
// bounds of the window in at most W - 1 buckets of B values (the last word counts those above the
// window) and keeps the bucket that holds the answer, until buckets are single values.  If bounds
// fell between passes so that not even lo qualifies any more, lo is returned: still a bound (the
// h-index of the values read is below it), and the neighbour that fell schedules v again.
template <unsigned G, uint32_t W>
__device__ uint32_t grp_hindex(uint32_t b, uint32_t e, uint32_t hv, const uint32_t *__restrict__ col,
                               const uint32_t *__restrict__ h, uint32_t *hist, unsigned gl, unsigned *s_red) {
    uint32_t lo = 0, top = hv;
    while (true) {
        const uint32_t size = top - lo + 1;
        const uint32_t B = (uint32_t)(((uint64_t)size + (W - 2)) / (W - 1));
        const uint32_t nb = (size + B - 1) / B;   // <= W - 1
        grp_sync<G>();
        for (uint32_t i = gl; i <= nb; i += G) hist[i] = 0;
        grp_sync<G>();
        for (uint32_t j = b + gl; j < e; j += G) {
            const uint32_t y = min(h[col[j]], hv);
            if (y > top) atomicAdd(&hist[nb], 1u);
            else if (y >= lo) atomicAdd(&hist[(y - lo) / B], 1u);
        }
        grp_sync<G>();
        const uint32_t above = hist[nb];
        const unsigned c = grp_prefix_true<G>(hist, nb, above, lo, B, gl, s_red);
        const uint32_t i = c > 0 ? c - 1 : 0;
        if (B == 1) return lo + i;
        lo += i * B;
        top = min(lo + B - 1, top);
    }
}

// number of row entries [b, e) whose bound is >= k (one lane)
__device__ __forceinline__ uint32_t lane_count_ge(const uint32_t *__restrict__ col, const uint32_t *__restrict__ h,
                                                  uint32_t b, uint32_t e, uint32_t k) {
    uint32_t c = 0;
    for (uint32_t j = b; j < e; ++j) c += h[col[j]] >= k;
    return c;
}

// h-index of a lane's vertex, capped at hv: the count c of bounds >= hv is a lower bound, and
// binary search over [c, hv - 1] finds the largest k with at least k bounds >= k
__device__ __forceinline__ uint32_t lane_hindex(uint32_t b, uint32_t e, uint32_t hv, const uint32_t *__restrict__ col,
                                                const uint32_t *__restrict__ h) {
    if (hv == 0) return 0;
    const uint32_t c = lane_count_ge(col, h, b, e, hv);
    if (c >= hv) return hv;
    uint32_t lo = c, hi = hv - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (lane_count_ge(col, h, b, e, mid) >= mid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct Ctx {
    const uint32_t *__restrict__ row;
    const uint32_t *__restrict__ col;
    uint32_t *__restrict__ h;       // bounds, then core numbers
    uint32_t *__restrict__ d;       // neighbours of core >= own, not yet removed
    uint32_t *__restrict__ rnd;     // removal round
    uint32_t *__restrict__ mark;    // phase a vertex is to be processed in (h-index stage)
    CoreCtl *__restrict__ ctl;
    unsigned *s_flag;               // LDS: this block scheduled work for the next phase
};

// --- the three stages' work on one vertex, for a lane, a wavefront or the workgroup -------------

// h-index stage: lower h(v), and schedule for phase `next` the neighbours whose bound is above the
// new value (a plain store: every writer writes the same tag)
__device__ __forceinline__ void schedule(uint32_t w, uint32_t nh, uint32_t next, const Ctx &C) {
    if (C.h[w] > nh && C.mark[w] != next) {
        C.mark[w] = next;
        *C.s_flag = 1;
    }
}

template <unsigned G, uint32_t W>
__device__ void grp_hindex_vertex(uint32_t v, const Ctx &C, uint32_t next, unsigned gl, uint32_t *hist,
                                  unsigned *s_red) {
    const uint32_t b = C.row[v], e = C.row[v + 1];
    const uint32_t hv = C.h[v];   // written only by v's own processing
    if (hv == 0) return;
    const uint32_t nh = grp_hindex<G, W>(b, e, hv, C.col, C.h, hist, gl, s_red);
    if (nh >= hv) return;
    if (gl == 0) __hip_atomic_store(&C.h[v], nh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t j = b + gl; j < e; j += G) schedule(C.col[j], nh, next, C);
}

__device__ void lane_hindex_vertex(uint32_t v, const Ctx &C, uint32_t next) {
    const uint32_t b = C.row[v], e = C.row[v + 1];
    const uint32_t hv = C.h[v];
    const uint32_t nh = lane_hindex(b, e, hv, C.col, C.h);
    if (nh >= hv) return;
    __hip_atomic_store(&C.h[v], nh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t j = b; j < e; ++j) schedule(C.col[j], nh, next, C);
}

// degree stage: d(v) = neighbours of core >= core(v); d(v) <= core(v) puts v in removal round 0
__device__ __forceinline__ void degree_done(uint32_t v, uint32_t dv, uint32_t hv, const Ctx &C, unsigned *s_kappa) {
    C.d[v] = dv;
    if (dv < hv) atomicOr(&C.ctl->error, 4u);   // no vertex has fewer such neighbours than its core
    if (dv <= hv) {
        C.rnd[v] = 0;
        *C.s_flag = 1;
    }
    atomicMax(s_kappa, hv);
}

template <unsigned G>
__device__ void grp_degree_vertex(uint32_t v, const Ctx &C, unsigned gl, unsigned *s_red, unsigned *s_kappa) {
    const uint32_t b = C.row[v], e = C.row[v + 1];
    const uint32_t hv = C.h[v];
    unsigned c = 0;
    for (uint32_t j = b + gl; j < e; j += G) c += C.h[C.col[j]] >= hv;
    c = grp_sum<G>(c, s_red);
    if (gl == 0) degree_done(v, c, hv, C, s_kappa);
}

__device__ void lane_degree_vertex(uint32_t v, const Ctx &C, unsigned *s_kappa) {
    const uint32_t hv = C.h[v];
    degree_done(v, lane_count_ge(C.col, C.h, C.row[v], C.row[v + 1], hv), hv, C, s_kappa);
}

// removal stage, round r: v leaves its shell; a shell neighbour not yet removed whose d falls from
// core + 1 to core is removed in round r + 1 (d only falls, once per removed neighbour, so exactly
// one decrement sees core + 1)
__device__ __forceinline__ void remove_edge(uint32_t w, uint32_t cv, uint32_t r, const Ctx &C) {
    if (C.h[w] != cv || C.rnd[w] != kUnset) return;
    if (atomicSub(&C.d[w], 1u) != cv + 1) return;
    C.rnd[w] = r + 1;
    *C.s_flag = 1;
}

template <unsigned G>
__device__ void grp_remove_vertex(uint32_t v, const Ctx &C, uint32_t r, unsigned gl) {
    const uint32_t b = C.row[v], e = C.row[v + 1];
    const uint32_t cv = C.h[v];
    for (uint32_t j = b + gl; j < e; j += G) remove_edge(C.col[j], cv, r, C);
}

__device__ void lane_remove_vertex(uint32_t v, const Ctx &C, uint32_t r) {
    const uint32_t b = C.row[v], e = C.row[v + 1];
    const uint32_t cv = C.h[v];
    for (uint32_t j = b; j < e; ++j) remove_edge(C.col[j], cv, r, C);
}

// Whether v is processed in this phase: in the h-index stage when scheduled for it or already for
// the next one (skipping those would let a vertex whose neighbours keep changing be put off phase
// after phase), in the removal stage when removed in this round, in the degree stage always.
template <int S>
__device__ __forceinline__ bool is_active(uint32_t v, uint32_t arg, const Ctx &C) {
    if constexpr (S == kHindex) return __hip_atomic_load(&C.mark[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= arg;
    else if constexpr (S == kRemove) return C.rnd[v] == arg;
    else return true;
}

// One phase over the vertex list `all` (grouped by row kind, each kind in vertex order), split
// statically: workgroup-kind vertices by block, wavefront-kind and lane-kind ones in chunks of 64
// by wavefront.  A group's decision to process a vertex is read once and shared, so that all of it
// takes the same branch.  arg: the phase (h-index), the round (removal).
template <int S>
__device__ void run_phase(const Ctx &C, const uint32_t *__restrict__ all, const uint32_t base[3],
                          const uint32_t cnt[3], uint32_t arg, uint32_t *s_hist, unsigned *s_red,
                          unsigned *s_item, unsigned *s_kappa) {
    const unsigned tid = threadIdx.x, lane = tid & 63, wave = tid / 64;
    const uint32_t gw = blockIdx.x * kWaves + wave, nw = gridDim.x * kWaves;
    for (uint32_t i = blockIdx.x; i < cnt[2]; i += gridDim.x) {
        const uint32_t v = all[base[2] + i];
        if (tid == 0) *s_item = is_active<S>(v, arg, C) ? 1u : 0u;
        __syncthreads();
        const bool act = *s_item != 0;
        __syncthreads();
        if (!act) continue;
        if constexpr (S == kHindex) grp_hindex_vertex<kBlock, kBlockHist>(v, C, arg + 1, tid, s_hist, s_red);
        else if constexpr (S == kDegree) grp_degree_vertex<kBlock>(v, C, tid, s_red, s_kappa);
        else grp_remove_vertex<kBlock>(v, C, arg, tid);
    }
    uint32_t *w_hist = s_hist + wave * kWaveHist;
    for (uint32_t c0 = gw * 64; c0 < cnt[1]; c0 += nw * 64) {
        const uint32_t i = c0 + lane;
        const uint32_t v = i < cnt[1] ? all[base[1] + i] : 0u;
        uint64_t m = __ballot(i < cnt[1] && is_active<S>(v, arg, C));
        while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const uint32_t u = __shfl(v, src, 64);
            if constexpr (S == kHindex) grp_hindex_vertex<64, kWaveHist>(u, C, arg + 1, lane, w_hist, nullptr);
            else if constexpr (S == kDegree) grp_degree_vertex<64>(u, C, lane, nullptr, s_kappa);
            else grp_remove_vertex<64>(u, C, arg, lane);
        }
    }
    for (uint32_t c0 = gw * 64; c0 < cnt[0]; c0 += nw * 64) {
        const uint32_t i = c0 + lane;
        if (i >= cnt[0]) continue;
        const uint32_t v = all[base[0] + i];
        if (!is_active<S>(v, arg, C)) continue;
        if constexpr (S == kHindex) lane_hindex_vertex(v, C, arg + 1);
        else if constexpr (S == kDegree) lane_degree_vertex(v, C, s_kappa);
        else lane_remove_vertex(v, C, arg);
    }
}

__global__ void __launch_bounds__(kBlock)
k_core(uint32_t n, uint64_t max_phases, const uint32_t *__restrict__ row, const uint32_t *__restrict__ col,
       uint32_t *__restrict__ h, uint32_t *__restrict__ d, uint32_t *__restrict__ rnd, uint32_t *__restrict__ mark,
       uint32_t *__restrict__ all, uint32_t *__restrict__ bcnt, CoreCtl *__restrict__ ctl) {
    __shared__ __attribute__((aligned(16))) uint32_t s_hist[kBlockHist];
    __shared__ unsigned s_red[kWaves], s_item, s_flag, s_kappa, s_cls[3], s_wc[kWaves][3];
    const unsigned tid = threadIdx.x, lane = tid & 63, wave = tid / 64;
    const uint64_t below = (1ull << lane) - 1;
    unsigned target = 0;
    const Ctx C{row, col, h, d, rnd, mark, ctl, &s_flag};
    // each block sets up a contiguous range of vertices
    const uint32_t chunk = (uint32_t)((((uint64_t)n + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock);
    const uint32_t v_lo = (uint32_t)min((uint64_t)blockIdx.x * chunk, (uint64_t)n);
    const uint32_t v_hi = (uint32_t)min((uint64_t)v_lo + chunk, (uint64_t)n);

    // setup: bounds start at the degrees; count the rows of each kind per block
    if (tid < 3) s_cls[tid] = 0;
    __syncthreads();
    for (uint32_t v = v_lo + tid; v < v_hi; v += kBlock) {
        const uint32_t len = row[v + 1] - row[v];
        h[v] = len;
        mark[v] = 0;   // every vertex is processed in phase 0
        rnd[v] = kUnset;
        atomicAdd(&s_cls[row_class(len)], 1u);
    }
    __syncthreads();
    if (tid < 3) bcnt[blockIdx.x * 3 + tid] = s_cls[tid];
    grid_barrier(ctl, target);
    if (ld_relaxed(&ctl->error)) return;
    // the list `all`: vertices grouped by row kind, in vertex order within a kind
    if (tid < 3) {   // this block's offset in each kind, and the kind's size
        uint32_t tot = 0, before = 0;
        for (uint32_t b = 0; b < gridDim.x; ++b) {
            const uint32_t x = ld_relaxed(&bcnt[b * 3 + tid]);
            tot += x;
            if (b < blockIdx.x) before += x;
        }
        s_wc[0][tid] = tot;
        s_wc[1][tid] = before;
    }
    __syncthreads();
    uint32_t cnt[3], off[3], base[3];
    for (int c = 0; c < 3; ++c) {
        cnt[c] = s_wc[0][c];
        off[c] = s_wc[1][c];
    }
    __syncthreads();
    base[0] = 0;
    base[1] = cnt[0];
    base[2] = cnt[0] + cnt[1];
    for (uint32_t v0 = v_lo; v0 < v_hi; v0 += kBlock) {
        const uint32_t v = v0 + tid;
        const uint32_t cls = v < v_hi ? row_class(row[v + 1] - row[v]) : 3u;
        uint64_t m[3];
        for (int c = 0; c < 3; ++c) m[c] = __ballot(cls == (uint32_t)c);
        if (lane == 0)
            for (int c = 0; c < 3; ++c) s_wc[wave][c] = (unsigned)__popcll(m[c]);
        __syncthreads();
        for (int c = 0; c < 3; ++c) {
            uint32_t before = 0, tot = 0;
            for (unsigned w = 0; w < kWaves; ++w) {
                const unsigned x = s_wc[w][c];
                if (w < wave) before += x;
                tot += x;
            }
            if (cls == (uint32_t)c) {
                const uint32_t pos = off[c] + before + (uint32_t)__popcll(m[c] & below);
                if (pos < cnt[c]) all[base[c] + pos] = v;
                else atomicOr(&ctl->error, 2u);
            }
            off[c] += tot;
        }
        __syncthreads();
    }
    grid_barrier(ctl, target);
    if (ld_relaxed(&ctl->error)) return;

    // flags of phases mod 3: set when a phase schedules work for the next one; the flag of the
    // phase after next is cleared (no block reads it any more: it was the previous phase's)
    auto begin_phase = [&](uint64_t p) {
        if (blockIdx.x == 0 && tid == 0) ctl->flag[(p + 2) % 3] = 0;
        if (tid == 0) s_flag = 0;
        __syncthreads();
    };
    auto end_phase = [&](uint64_t p) {
        __syncthreads();
        if (tid == 0 && s_flag) __hip_atomic_store(&ctl->flag[(p + 1) % 3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        grid_barrier(ctl, target);
        return ld_relaxed(&ctl->error) == 0;
    };
    uint64_t p = 0;
    // stage 1: h-index phases until one schedules nothing
    while (true) {
        if (p >= max_phases) {
            if (blockIdx.x == 0 && tid == 0) atomicOr(&ctl->error, 8u);
            return;
        }
        begin_phase(p);
        run_phase<kHindex>(C, all, base, cnt, (uint32_t)p, s_hist, s_red, &s_item, &s_kappa);
        if (!end_phase(p)) return;
        const bool more = ld_relaxed(&ctl->flag[(p + 1) % 3]) != 0;
        ++p;
        if (!more) break;
    }
    if (blockIdx.x == 0 && tid == 0) ctl->iters = (unsigned)p;
    // stage 2a: d(v) for every vertex, and removal round 0
    if (tid == 0) s_kappa = 0;
    begin_phase(p);
    run_phase<kDegree>(C, all, base, cnt, 0u, s_hist, s_red, &s_item, &s_kappa);
    __syncthreads();
    if (tid == 0 && s_kappa) atomicMax(&ctl->kappa, s_kappa);
    if (!end_phase(p)) return;
    bool more = ld_relaxed(&ctl->flag[(p + 1) % 3]) != 0;
    ++p;
    // stage 2b: removal rounds
    uint32_t r = 0;
    while (more) {
        if (p >= max_phases) {
            if (blockIdx.x == 0 && tid == 0) atomicOr(&ctl->error, 8u);
            return;
        }
        begin_phase(p);
        run_phase<kRemove>(C, all, base, cnt, r, s_hist, s_red, &s_item, &s_kappa);
        if (!end_phase(p)) return;
        more = ld_relaxed(&ctl->flag[(p + 1) % 3]) != 0;
        ++p;
        ++r;
    }
    if (blockIdx.x == 0 && tid == 0) ctl->rounds = r;
    // every vertex must have been removed
    for (uint32_t v = v_lo + tid; v < v_hi; v += kBlock)
        if (rnd[v] == kUnset) atomicOr(&ctl->error, 16u);
}

__global__ void k_order_keys(uint32_t n, uint32_t rbits, const uint32_t *__restrict__ core,
                             const uint32_t *__restrict__ rnd, uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
    const uint32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    key[v] = ((uint64_t)core[v] << rbits) | rnd[v];
    val[v] = v;
}

__global__ void k_rank_of(uint32_t n, const uint32_t *__restrict__ order, uint32_t *__restrict__ rank) {
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    if (p < n) rank[order[p]] = p;
}

uint32_t bits_for(uint64_t x) {   // bits to hold values 0..x
    uint32_t b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

}  // namespace

int core_order(dt_graph *g) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    DT_TRY(dev_alloc(ctx, g->core, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->order, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->rank, (uint64_t)n * 4));
    if (n == 0) {
        g->kappa = 0;
        g->peel_rounds = 0;
        return DT_OK;
    }
    DevMem dm, rndm, markm, allm, bcm, ctlm;
    DT_TRY(dev_alloc(ctx, dm, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, rndm, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, markm, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, allm, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, ctlm, sizeof(CoreCtl)));
    int per_cu = 0;
    DT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_core, kBlock, 0));
    if (per_cu <= 0) return fail(DT_EDEVICE, "core kernel cannot be resident");
    unsigned grid = (unsigned)ctx->num_cus;
    const unsigned want = grid_for(n, kBlock);
    if (want < grid) grid = want;
    if (grid > (unsigned)ctx->num_cus * (unsigned)per_cu) grid = (unsigned)ctx->num_cus * (unsigned)per_cu;
    DT_TRY(dev_alloc(ctx, bcm, (uint64_t)grid * 3 * 4));
    DT_HIP(hipMemsetAsync(ctlm.ptr, 0, sizeof(CoreCtl), st));
    // both stages together: every bound falls at most 2 m_s times in all, and every round removes
    // at least one vertex
    uint64_t max_phases = 2ull * g->m_s + 2ull * n + 8;
    const uint32_t *row = g->row.as<uint32_t>(), *col = g->col.as<uint32_t>();
    uint32_t *h = g->core.as<uint32_t>(), *d = dm.as<uint32_t>(), *rnd = rndm.as<uint32_t>(),
             *mark = markm.as<uint32_t>(), *all = allm.as<uint32_t>(), *bcnt = bcm.as<uint32_t>();
    CoreCtl *ctl = ctlm.as<CoreCtl>();
    uint32_t nn = n;
    void *args[] = {&nn, &max_phases, &row, &col, &h, &d, &rnd, &mark, &all, &bcnt, &ctl};
    prof_begin(ctx, kProfCore, st);
    DT_HIP(hipLaunchCooperativeKernel((const void *)k_core, dim3(grid), dim3(kBlock), args, 0, st));
    prof_end(ctx, kProfCore, st);
    CoreCtl hc{};
    DT_HIP(hipMemcpyAsync(&hc, ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    if (hc.error & 1u) return fail(DT_EDEVICE, "core ordering barrier timed out");
    if (hc.error) return fail(DT_EDEVICE, "core ordering failed its consistency checks (code %u)", hc.error);
    g->kappa = hc.kappa;
    g->peel_rounds = hc.iters + hc.rounds;
    g->alg_bytes_peel = 16ull * n + 16ull * g->m_s;
    // the ordering: by (core, round)
    const uint32_t rb = bits_for(hc.rounds), cb = bits_for(hc.kappa);
    DevMem kin, kout, vin;
    DT_TRY(dev_alloc(ctx, kin, (uint64_t)n * 8));
    DT_TRY(dev_alloc(ctx, kout, (uint64_t)n * 8));
    DT_TRY(dev_alloc(ctx, vin, (uint64_t)n * 4));
    k_order_keys<<<grid_for(n, 256), 256, 0, st>>>(n, rb, h, rnd, kin.as<uint64_t>(), vin.as<uint32_t>());
    DT_HIP(hipGetLastError());
    const int end_bit = (int)(rb + cb) > 0 ? (int)(rb + cb) : 1;
    DT_TRY(sort_pairs_u64_u32(ctx, kin.as<uint64_t>(), kout.as<uint64_t>(), vin.as<uint32_t>(),
                              g->order.as<uint32_t>(), n, end_bit, st));
    k_rank_of<<<grid_for(n, 256), 256, 0, st>>>(n, g->order.as<uint32_t>(), g->rank.as<uint32_t>());
    DT_HIP(hipGetLastError());
    DT_HIP(hipStreamSynchronize(st));
    return DT_OK;
}

int order_vertices(dt_graph *g) { return g->tuning.order_method == 1 ? core_order(g) : peel(g); }

}  // namespace dt
