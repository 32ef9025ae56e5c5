// Degeneracy ordering by a parallel k-core peel (Section 3, the degeneracy ordering: vertices taken
// in order of smallest remaining degree; the degeneracy is the largest core number).
//
// Level k removes every remaining vertex whose remaining degree is <= k: the vertices found by a
// scan of the remaining ones, then those whose degree falls to k while their neighbours are
// removed.  A vertex takes its position in the ordering no later than the start of its own
// removal, and positions are handed out in time order.  When v is queued at most k of its
// neighbours are not yet removed; a neighbour placed after v started its removal after v was
// placed, hence after v was queued, so it is one of those: the out-degree of v in G_prec is at
// most k = core(v) <= degeneracy, the property Theorem 1's bound rests on.  (Different removal
// orders give different orientations but the same counts: each static triangle is counted once
// under its own naming u < v < w.)
//
// The whole peel is one cooperative (co-resident) grid: levels and rounds are separated by grid
// barriers instead of kernel launches and host round trips, since power-law graphs need thousands
// of removal steps, most with frontiers of a few vertices.  Within a level, a block removes the
// vertices its own removals queued right away (a cascade local to the block, with workgroup
// barriers only), so a grid round usually ends a level; only vertices queued past a full staging
// list wait for another round.  The first levels remove most of the graph and are bound by work,
// the later ones by latency, and a barrier's cost grows with the number of blocks that meet at it:
// the grid starts with one block of 1024 threads per CU and narrows to 128, 64, then 32 blocks
// as vertices run out.  The barrier is a monotonic arrival counter that every block polls.  Counters
// that decide the next step (queue positions taken in a phase, survivors of a level scan) rotate
// over three slots, so a fast block starting the next phase never changes what a slow block reads,
// and every block takes the same branch.  A vertex is queued at most
// once: by the level scan when its degree is <= k (no decrement runs during a scan), or by the
// single decrement that takes its degree from k + 1 to k (degrees only fall, and a queued vertex
// already has degree <= k, so no later decrement can see k + 1 again); a vertex queued by a
// decrement also gets a large negative degree, so that the next scans, which still list it, skip
// it.  The queue index is also bounds-checked, and the host checks that exactly n vertices were
// queued.  A barrier that waits far longer than any peel could take sets an error flag and lets its
// block go, so that a fault in this logic ends the kernel instead of hanging it.
#include "internal.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 1024;
constexpr unsigned kGridWide = 256;    // blocks of the first levels
// the grid narrows as vertices run out: blocks while at least `from` vertices remain (timed per
// phase on the 61M-edge graph: one width for all of them below 200,000 vertices, 16 or 8 blocks
// there, and 256 blocks down to 16,000 vertices were all slower)
struct Width {
    uint32_t from;
    unsigned blocks;
};
constexpr Width kWidths[4] = {{1000000, kGridWide}, {200000, 128}, {50000, 64}, {0, 32}};
constexpr uint32_t kTail = kPeelTailMax;   // most vertices the one-workgroup finish takes (16-bit ids)
// LDS of a peel block.  The one-workgroup finish keeps there the local CSR rows (kTail + 1
// words), the degrees (16-bit, two per word), the removal queue and the list of vertices not yet
// queued (16-bit local ids); on the grid the same words stage the vertices a block queues in one
// round.
constexpr uint32_t kRowWords = kTail + 1, kDegWords = kTail / 2, kQWords = kTail / 2, kLiveWords = kTail / 2;
constexpr uint32_t kLdsWords = kRowWords + kDegWords + kQWords + kLiveWords;
// on the grid the words hold two staging halves: the vertices a block is removing and those their
// removal queues
constexpr uint32_t kStage = kLdsWords / 2;
constexpr uint32_t kUnset = 0xffffffffu;
constexpr long kSpinLimit = 1l << 26;
// degree of a vertex queued during removal rounds: negative, and it stays negative under the
// at most n further decrements, so a level scan never takes it again
constexpr int kRemoved = -(1 << 30);

struct PeelCtl {
    unsigned int qtail;      // vertices queued in all (written at the end)
    unsigned int qc[3];      // per grid phase mod 3: queue positions taken in that phase
    unsigned int ovc[3];     // per grid phase mod 3: vertices that phase queued past a full stage
    unsigned int arrived;    // barrier arrivals (only ever increases)
    unsigned int error;      // a barrier gave up waiting, or a consistency check failed
    unsigned int rounds;     // removal rounds
    unsigned int kappa;      // largest level that removed a vertex
    unsigned int nlvl;       // levels recorded by the one-workgroup finish
    unsigned long long lres; // hand-over: local ids (low word) and adjacency entries (high word) given out
    unsigned int ho;         // 1: the grid handed its last vertices over (the state below is set)
    unsigned int ho_tail, ho_k, ho_rounds;   // queue positions taken, level and rounds at the hand-over
    unsigned int scan[3][2]; // per level mod 3: survivors of the level scan, their smallest degree
};

__device__ __forceinline__ unsigned ld_relaxed(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier.  Arrivals only ever increase, and every block passes the same barriers in the same
// order with the same participants, so a barrier is complete once `target` arrivals (the running
// sum of the participants of every barrier so far) have been counted: each block's first thread
// publishes its block's writes, arrives, and polls the count; no block has to release the others.
// A barrier that waits far longer than any peel could take sets an error flag and lets its block
// go.
__device__ void grid_barrier(PeelCtl *ctl, unsigned target) {
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

// A vertex whose degree a removal took from k + 1 to k joins the block's staging list, which the
// same block removes next (its position in the ordering is taken then); a full staging list sends
// the rest to the overflow list, which the next grid phase takes.
__device__ __forceinline__ void enqueue(uint32_t v, uint32_t k, uint32_t n, uint32_t *level, int *deg,
                                        unsigned *ovc, uint32_t *ovf, unsigned *err, uint32_t *s_stage,
                                        unsigned *s_cnt) {
    level[v] = k;
    __hip_atomic_store(&deg[v], kRemoved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t p = atomicAdd(s_cnt, 1u);
    if (p < kStage) {
        s_stage[p] = v;
    } else {
        const uint32_t o = atomicAdd(ovc, 1u);
        if (o < n) ovf[o] = v;
        else atomicOr(err, 8u);
    }
}

__device__ __forceinline__ unsigned wave_min(unsigned x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    return x;
}

// remove the adjacency entries [b, e) of one vertex (this lane: first, first + stride, ...)
__device__ __forceinline__ void remove_range(uint32_t b, uint32_t e, uint32_t first, uint32_t stride, uint32_t k,
                                             uint32_t n, const uint32_t *__restrict__ col, int *__restrict__ deg,
                                             uint32_t *__restrict__ level, unsigned *ovc, uint32_t *ovf,
                                             unsigned *err, uint32_t *s_stage, unsigned *s_cnt) {
    uint32_t j = b + first;
    // four independent decrements in flight per lane
    for (; j + 3 * stride < e; j += 4 * stride) {
        const uint32_t x0 = col[j], x1 = col[j + stride], x2 = col[j + 2 * stride], x3 = col[j + 3 * stride];
        const int o0 = atomicSub(&deg[x0], 1), o1 = atomicSub(&deg[x1], 1), o2 = atomicSub(&deg[x2], 1),
                  o3 = atomicSub(&deg[x3], 1);
        if (o0 == (int)k + 1) enqueue(x0, k, n, level, deg, ovc, ovf, err, s_stage, s_cnt);
        if (o1 == (int)k + 1) enqueue(x1, k, n, level, deg, ovc, ovf, err, s_stage, s_cnt);
        if (o2 == (int)k + 1) enqueue(x2, k, n, level, deg, ovc, ovf, err, s_stage, s_cnt);
        if (o3 == (int)k + 1) enqueue(x3, k, n, level, deg, ovc, ovf, err, s_stage, s_cnt);
    }
    for (; j < e; j += stride) {
        const uint32_t x = col[j];
        const int old = atomicSub(&deg[x], 1);
        if (old == (int)k + 1) enqueue(x, k, n, level, deg, ovc, ovf, err, s_stage, s_cnt);
    }
}

__device__ __forceinline__ void remove_edges(uint32_t v, uint32_t first, uint32_t stride, uint32_t k,
                                             uint32_t n, const uint32_t *__restrict__ row,
                                             const uint32_t *__restrict__ col, int *__restrict__ deg,
                                             uint32_t *__restrict__ level, unsigned *ovc, uint32_t *ovf,
                                             unsigned *err, uint32_t *s_stage, unsigned *s_cnt) {
    remove_range(row[v], row[v + 1], first, stride, k, n, col, deg, level, ovc, ovf, err, s_stage, s_cnt);
}

// The last vertices: one workgroup finishes the peel on the subgraph they induce, with local
// (16-bit) vertex ids.  The local CSR rows, the degrees, the removal queue and the list of vertices
// not yet queued live in LDS, so a round touches global memory only to read adjacency (lcol);
// workgroup barriers separate rounds.  rlist maps local ids to vertices.  A degree counts the
// neighbours not yet removed (so it never falls below zero, and two 16-bit degrees share a word
// safely) until the vertex is queued; queuing adds kMark - degree, which puts it at kMark, and
// the at most kTail later decrements leave it at least kMark - kTail, above every level.  Each
// wavefront keeps its own segment of the live list and compacts it in place at every level scan,
// so a scan reads only the vertices still live, and takes one atomic per wavefront for the
// survivors' count and smallest degree.  The queue positions (continuing from qbase) and the core
// numbers are written at the end, from the queue and the level boundaries recorded in lvl (pairs:
// first queue position, level).
constexpr uint32_t kMark = 0xC000u, kMarked = 0x8000u;
static_assert(kMark - kTail > kMarked && kMarked > kTail, "queued degrees stay above every level");
__device__ void peel_tail(uint32_t R, uint32_t qbase, uint32_t k, uint32_t rounds,
                          const uint32_t *__restrict__ rlist, const uint32_t *__restrict__ lrow,
                          const uint16_t *__restrict__ lcol, uint32_t *__restrict__ lvl,
                          uint32_t *__restrict__ level, uint32_t *__restrict__ queue, PeelCtl *ctl,
                          uint32_t *s_mem) {
    uint32_t *s_row = s_mem;                                              // kRowWords
    uint32_t *s_deg = s_mem + kRowWords;                                  // kDegWords
    uint16_t *s_q = reinterpret_cast<uint16_t *>(s_mem + kRowWords + kDegWords);               // kTail
    uint16_t *s_live = reinterpret_cast<uint16_t *>(s_mem + kRowWords + kDegWords + kQWords);  // kTail
    __shared__ unsigned s_qt, s_keep, s_min, s_nlvl;
    const unsigned tid = threadIdx.x, lane = tid & 63, wave = tid / 64;
    constexpr unsigned kWaves = kBlock / 64;
    const uint64_t below = (1ull << lane) - 1;
    for (uint32_t l = tid; l <= R; l += kBlock) s_row[l] = lrow[l];
    for (uint32_t w = tid; w < kDegWords; w += kBlock) s_deg[w] = 0;
    for (uint32_t l = tid; l < R; l += kBlock) s_live[l] = (uint16_t)l;
    __syncthreads();
    for (uint32_t l = tid; l < R; l += kBlock)
        atomicAdd(&s_deg[l >> 1], (s_row[l + 1] - s_row[l]) << ((l & 1) * 16));
    if (tid == 0) {
        s_qt = 0;
        s_nlvl = 0;
    }
    // this wavefront's segment of the live list: [lb, lb + lc)
    const uint32_t seg = (R + kWaves - 1) / kWaves;
    const uint32_t lb = wave * seg < R ? wave * seg : R;
    uint32_t lc = (lb + seg < R ? lb + seg : R) - lb;
    uint32_t h = 0, t = 0;
    auto deg_of = [&](uint32_t l) { return (s_deg[l >> 1] >> ((l & 1) * 16)) & 0xffffu; };
    // queue y, whose degree is d (no decrement of y runs between reading d and this)
    auto mark = [&](uint32_t y, uint32_t d) { atomicAdd(&s_deg[y >> 1], (kMark - d) << ((y & 1) * 16)); };
    // remove one edge end at y; a degree taken from k + 1 to k queues y
    auto dec = [&](uint32_t y, uint32_t kk) {
        const uint32_t sh = (y & 1) * 16;
        const uint32_t old = (atomicSub(&s_deg[y >> 1], 1u << sh) >> sh) & 0xffffu;
        if (old == kk + 1) {
            atomicAdd(&s_deg[y >> 1], (kMark - kk) << sh);
            const uint32_t p = atomicAdd(&s_qt, 1u);
            if (p < R) s_q[p] = (uint16_t)y;
        }
    };
    while (true) {
        __syncthreads();
        if (tid == 0) {
            s_keep = 0;
            s_min = 0xffffffffu;
        }
        __syncthreads();
        const uint32_t level_start = t;
        // level scan over this wavefront's live vertices: queue those of degree <= k, keep the
        // others (written back in place: a survivor's new slot is never after its old one, and
        // the wavefront reads a chunk before it writes any of it)
        {
            uint32_t nk = 0;
            unsigned md = 0xffffffffu;
            for (uint32_t i0 = 0; i0 < lc; i0 += 64) {
                const uint32_t i = i0 + lane;
                uint32_t l = 0, d = kMark;
                if (i < lc) {
                    l = s_live[lb + i];
                    d = deg_of(l);
                }
                const bool tk = d <= k, kp = d > k && d < kMarked;
                const uint64_t mt = __ballot(tk), mk = __ballot(kp);
                if (mt) {
                    uint32_t qb = 0;
                    if (lane == 0) qb = atomicAdd(&s_qt, (unsigned)__popcll(mt));
                    qb = __shfl(qb, 0, 64);
                    if (tk) {
                        const uint32_t p = qb + (uint32_t)__popcll(mt & below);
                        mark(l, d);
                        if (p < R) s_q[p] = (uint16_t)l;
                    }
                }
                if (kp) {
                    s_live[lb + nk + (uint32_t)__popcll(mk & below)] = (uint16_t)l;
                    md = d < md ? d : md;
                }
                nk += (uint32_t)__popcll(mk);
            }
            lc = nk;
            md = wave_min(md);
            if (lane == 0 && nk) {
                atomicAdd(&s_keep, nk);
                atomicMin(&s_min, md);
            }
        }
        __syncthreads();
        t = s_qt;
        const uint32_t keep = s_keep, md = s_min;
        if (keep == 0) h = t;   // every remaining vertex is queued: nothing left to update
        // rounds: remove s_q[h, t)
        while (h < t) {
            const uint32_t f = t - h;
            uint32_t i0, first, stride, step;
            if (f >= kWaves) {
                i0 = h + wave; first = lane; stride = 64; step = kWaves;
            } else {
                const uint32_t per = kWaves / f;
                i0 = h + wave / per; first = (wave % per) * 64 + lane; stride = per * 64; step = f;
                if (wave / per >= f) i0 = t;
            }
            for (uint32_t i = i0; i < t; i += step) {
                const uint32_t x = s_q[i];
                const uint32_t e = s_row[x + 1];
                uint32_t j = s_row[x] + first;
                for (; j + 3 * stride < e; j += 4 * stride) {
                    const uint32_t y0 = lcol[j], y1 = lcol[j + stride], y2 = lcol[j + 2 * stride],
                                   y3 = lcol[j + 3 * stride];
                    dec(y0, k);
                    dec(y1, k);
                    dec(y2, k);
                    dec(y3, k);
                }
                for (; j < e; j += stride) dec(lcol[j], k);
            }
            ++rounds;
            __syncthreads();
            h = t;
            t = s_qt;
            __syncthreads();
        }
        if (t > level_start && tid == 0) {   // this level removed s_q[level_start, t)
            const uint32_t li = s_nlvl++;
            lvl[2 * li] = level_start;
            lvl[2 * li + 1] = k;
        }
        if (t >= R) break;
        uint32_t next = k + 1;
        if (t == level_start && md != 0xffffffffu && md > next) next = md;
        k = next;
        if (k > R + qbase + 1) {   // cannot happen, as in the grid loop
            if (tid == 0) atomicOr(&ctl->error, 2u);
            break;
        }
    }
    __syncthreads();
    // queue positions and core numbers of the removed vertices, in removal order
    const uint32_t nl = s_nlvl, nq = t < R ? t : R;
    __threadfence_block();
    for (uint32_t p = tid; p < nq; p += kBlock) {
        const uint32_t v = rlist[s_q[p]];
        queue[qbase + p] = v;
        uint32_t lo = 0, len = nl;   // last boundary at or before p
        while (len > 0) {
            const uint32_t half = len >> 1;
            if (lvl[2 * (lo + half)] <= p) {
                lo += half + 1;
                len -= half + 1;
            } else {
                len = half;
            }
        }
        level[v] = lo > 0 ? lvl[2 * (lo - 1) + 1] : k;
    }
    if (tid == 0) {
        __hip_atomic_store(&ctl->qtail, qbase + nq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ctl->kappa = k;
        ctl->rounds = rounds;
        ctl->nlvl = nl;
    }
}

__global__ void __launch_bounds__(kBlock)
k_peel(uint32_t n, const uint32_t *__restrict__ row, const uint32_t *__restrict__ col,
       int *__restrict__ deg, uint32_t *__restrict__ level, uint32_t *__restrict__ queue,
       uint32_t *__restrict__ alive_a, uint32_t *__restrict__ alive_b, uint32_t *__restrict__ loc,
       uint32_t *__restrict__ rlist, uint32_t *__restrict__ lrow, uint32_t *__restrict__ lvl,
       uint16_t *__restrict__ lcol, uint64_t lcol_cap, uint32_t tail_cap, uint32_t *__restrict__ ovf0,
       uint32_t *__restrict__ ovf1, PeelCtl *__restrict__ ctl) {
    // the whole grid takes part while many vertices remain, then ever fewer of its first blocks
    unsigned nblk = gridDim.x;
    const uint32_t gtid = blockIdx.x * kBlock + threadIdx.x;
    uint32_t gsize = nblk * kBlock;
    const uint32_t gwave = gtid / 64, lane = threadIdx.x & 63;
    uint32_t nwaves = gsize / 64;
    const uint64_t below = (1ull << lane) - 1;
    unsigned btarget = 0;   // arrivals that complete the next barrier, less its participants
    __shared__ __attribute__((aligned(16))) uint32_t s_mem[kLdsWords];
    __shared__ unsigned s_cnt, s_base;
    __shared__ unsigned s_wct[kBlock / 64], s_wck[kBlock / 64], s_wmd[kBlock / 64], s_bq, s_bk;

    // the host cleared the control block; initialise per-vertex state
    for (uint32_t v = gtid; v < n; v += gsize) {
        deg[v] = (int)(row[v + 1] - row[v]);
        level[v] = kUnset;
        alive_a[v] = v;
        loc[v] = kUnset;
    }
    if (gtid == 0)
        for (int x = 0; x < 3; ++x) ctl->scan[x][1] = 0xffffffffu;
    grid_barrier(ctl, btarget += nblk);

    // tail: vertices queued before the current grid phase (a scan or a round); phase ph takes its
    // queue positions tail + [0, qc[ph % 3]) and every block adds the final count after the phase's
    // barrier, so all blocks agree on tail although a fast block may already be in the next phase
    uint32_t k = 0, head = 0, tail = 0, n_alive = n, prev_tail = 0, rounds = 0, lv = 0, ph = 0;
    uint32_t *cur = alive_a, *nxt = alive_b;
    bool done = false;
    // here every queued vertex has been removed: n - tail vertices remain
    while (n - tail > tail_cap) {
        // level scan: queue every remaining vertex of degree <= k, keep the others.  Each
        // wavefront takes a contiguous segment and counts its picks and survivors; its block
        // reserves room for all of them in both lists (one atomic each), and each wavefront then
        // writes its picks in order (no degree changes during a scan), so both lists keep the
        // roughly ascending vertex order of the previous one and the degree reads of the next scan
        // stay coalesced.
        {
            const uint32_t seg = ((n_alive + nwaves - 1) / nwaves + 63) & ~63u;
            const uint32_t sb = gwave * seg < n_alive ? gwave * seg : n_alive;
            const uint32_t se = sb + seg < n_alive ? sb + seg : n_alive;
            uint32_t ct = 0, ck = 0;
            unsigned mdl = 0xffffffffu;
            // four chunks of 64 at a time: their list reads, then their degree reads, in flight
            // together
            for (uint32_t b0 = sb; b0 < se; b0 += 4 * 64) {
                uint32_t vv[4];
                int dd[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t i = b0 + q * 64 + lane;
                    vv[q] = i < se ? cur[i] : 0u;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    dd[q] = b0 + q * 64 + lane < se ? ld_relaxed(&deg[vv[q]]) : -1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int d = dd[q];
                    const bool keep = d > (int)k;
                    ct += (uint32_t)__popcll(__ballot(d >= 0 && d <= (int)k));   // d < 0: queued
                    ck += (uint32_t)__popcll(__ballot(keep));
                    mdl = keep && (unsigned)d < mdl ? (unsigned)d : mdl;
                }
            }
            mdl = wave_min(mdl);
            // one reservation per block (the wavefronts' segments are consecutive, so a prefix
            // over them keeps the order): thousands of wavefronts meeting at the same counters
            // would serialise there
            const unsigned wv = threadIdx.x / 64;
            if (lane == 0) {
                s_wct[wv] = ct;
                s_wck[wv] = ck;
                s_wmd[wv] = mdl;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                unsigned tct = 0, tck = 0, bmd = 0xffffffffu;
                for (unsigned w = 0; w < kBlock / 64; ++w) {
                    const unsigned a = s_wct[w], b = s_wck[w];
                    s_wct[w] = tct;
                    s_wck[w] = tck;
                    tct += a;
                    tck += b;
                    bmd = s_wmd[w] < bmd ? s_wmd[w] : bmd;
                }
                s_bq = tct ? tail + atomicAdd(&ctl->qc[ph % 3], tct) : 0u;
                s_bk = tck ? atomicAdd(&ctl->scan[lv % 3][0], tck) : 0u;
                if (bmd != 0xffffffffu) atomicMin(&ctl->scan[lv % 3][1], bmd);
            }
            __syncthreads();
            uint32_t qb = s_bq + s_wct[wv], kb = s_bk + s_wck[wv];
            if (ct | ck) {
                for (uint32_t b0 = sb; b0 < se; b0 += 4 * 64) {
                    uint32_t vv[4];
                    int dd[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t i = b0 + q * 64 + lane;
                        vv[q] = i < se ? cur[i] : 0u;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        dd[q] = b0 + q * 64 + lane < se ? ld_relaxed(&deg[vv[q]]) : -1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t v = vv[q];
                        const int d = dd[q];
                        const bool take = d >= 0 && d <= (int)k, keep = d > (int)k;
                        const uint64_t mt = __ballot(take), mk = __ballot(keep);
                        if (take) {
                            level[v] = k;
                            const uint32_t p = qb + (uint32_t)__popcll(mt & below);
                            if (p < n) queue[p] = v;
                        }
                        if (keep) nxt[kb + (uint32_t)__popcll(mk & below)] = v;
                        qb += (uint32_t)__popcll(mt);
                        kb += (uint32_t)__popcll(mk);
                    }
                }
            }
        }
        grid_barrier(ctl, btarget += nblk);
        tail += ld_relaxed(&ctl->qc[ph % 3]);
        const uint32_t na2 = ld_relaxed(&ctl->scan[lv % 3][0]), md = ld_relaxed(&ctl->scan[lv % 3][1]);
        // the counters of the previous level were read by every block before this barrier: clear
        // them for the level after next (the next level's barrier publishes the clearing)
        if (gtid == 0) {
            __hip_atomic_store(&ctl->scan[(lv + 2) % 3][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->scan[(lv + 2) % 3][1], 0xffffffffu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->qc[(ph + 2) % 3], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->ovc[(ph + 2) % 3], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        ++lv;
        ++ph;
        // few vertices left: the later levels are latency-bound, and a barrier costs more the
        // more blocks meet at it, so the grid narrows in steps (only ever narrows)
        {
            unsigned want = kWidths[3].blocks;
            for (const Width &w : kWidths)
                if (na2 >= w.from) {
                    want = w.blocks;
                    break;
                }
            if (want < nblk) {
                if (blockIdx.x >= want) return;
                nblk = want;
                gsize = nblk * kBlock;
                nwaves = gsize / 64;
            }
        }
        // no survivors: every remaining vertex is queued at this level, and removing them can
        // queue nothing more
        if (na2 == 0) head = tail;
        // Rounds.  The frontier of the first is the scan's picks, queue[head, tail); each block
        // removes its share and then, without a grid barrier, removes the vertices that its own
        // removals queued (its staging list), step after step, until it queues nothing more; those
        // take their queue positions when their removal starts.  Only vertices queued past a full
        // staging list wait for the next round (overflow list; their positions are the round's
        // first).  A frontier of at least one vertex per wavefront is split by vertex; a smaller one
        // gives each vertex an equal share of the wavefronts.
        // Any order of removal within a level is a degeneracy ordering as long as every vertex
        // takes its position no later than its removal starts: a neighbour placed after it was not
        // yet removed when it was queued, so it counts among the at most k neighbours it had then.
        {
            uint32_t nf = tail - head;
            const uint32_t *fl = queue + head;
            bool first = true;
            while (nf > 0) {
                uint32_t *ovf_out = (ph & 1) ? ovf1 : ovf0;
                unsigned *ovc = &ctl->ovc[ph % 3];
                const uint32_t qbase = first ? tail : tail + nf;
                if (!first)
                    for (uint32_t i = gtid; i < nf; i += gsize)
                        if (tail + i < n) queue[tail + i] = fl[i];
                uint32_t *stage = s_mem, *front = s_mem + kStage;
                if (threadIdx.x == 0) s_cnt = 0;
                __syncthreads();
                if (nf >= nwaves) {
                    for (uint32_t i = gwave; i < nf; i += nwaves)
                        remove_edges(fl[i], lane, 64, k, n, row, col, deg, level, ovc, ovf_out, &ctl->error,
                                     stage, &s_cnt);
                } else {
                    const uint32_t per = nwaves / nf;
                    const uint32_t i = gwave / per, sub = gwave % per;
                    if (i < nf)
                        remove_edges(fl[i], sub * 64 + lane, per * 64, k, n, row, col, deg, level, ovc, ovf_out,
                                     &ctl->error, stage, &s_cnt);
                }
                // the block's own cascade
                for (uint32_t steps = 0;; ++steps) {
                    __syncthreads();
                    const uint32_t c = s_cnt < kStage ? s_cnt : kStage;
                    if (c == 0 || steps > n) break;
                    __syncthreads();
                    if (threadIdx.x == 0) {
                        s_base = qbase + atomicAdd(&ctl->qc[ph % 3], c);
                        s_cnt = 0;
                    }
                    uint32_t *t = stage;
                    stage = front;
                    front = t;
                    // this wavefront's first vertex and its adjacency bounds, read while the
                    // positions are being taken (reads only: its removal starts after them)
                    constexpr uint32_t kBW = kBlock / 64;
                    const uint32_t wave = threadIdx.x / 64;
                    const uint32_t per = c >= kBW ? 1 : kBW / c;
                    const uint32_t i0 = wave / per, sub = wave % per;
                    uint32_t rb = 0, re = 0;
                    if (i0 < c) {
                        const uint32_t v0 = front[i0];
                        rb = row[v0];
                        re = row[v0 + 1];
                    }
                    __syncthreads();
                    for (uint32_t x = threadIdx.x; x < c; x += kBlock) {
                        const uint32_t p = s_base + x;
                        if (p < n) queue[p] = front[x];
                    }
                    if (c >= kBW) {
                        if (i0 < c)
                            remove_range(rb, re, lane, 64, k, n, col, deg, level, ovc, ovf_out, &ctl->error, stage,
                                         &s_cnt);
                        for (uint32_t i = i0 + kBW; i < c; i += kBW)
                            remove_edges(front[i], lane, 64, k, n, row, col, deg, level, ovc, ovf_out, &ctl->error,
                                         stage, &s_cnt);
                    } else if (i0 < c) {
                        remove_range(rb, re, sub * 64 + lane, per * 64, k, n, col, deg, level, ovc, ovf_out,
                                     &ctl->error, stage, &s_cnt);
                    }
                }
                ++rounds;
                grid_barrier(ctl, btarget += nblk);
                tail = qbase + ld_relaxed(&ctl->qc[ph % 3]);
                head = tail;
                nf = ld_relaxed(ovc);
                fl = ovf_out;
                first = false;
                if (gtid == 0) {
                    __hip_atomic_store(&ctl->qc[(ph + 2) % 3], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&ctl->ovc[(ph + 2) % 3], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                ++ph;
                if (nf > n) {   // cannot happen: a vertex is queued once
                    if (gtid == 0) atomicOr(&ctl->error, 8u);
                    nf = 0;
                }
            }
        }
        if (tail >= n || ld_relaxed(&ctl->error)) {
            done = true;
            break;
        }
        // every survivor now has degree > k; when this level removed nothing, no degree changed
        // since the scan, so the smallest survivor degree is the next level that removes anything
        uint32_t next = k + 1;
        if (tail == prev_tail && md != 0xffffffffu && md > next) next = md;
        prev_tail = tail;
        k = next;
        if (k > n + 1) {   // cannot happen: some vertex is removed at the smallest survivor degree
            if (gtid == 0) atomicOr(&ctl->error, 2u);
            done = true;
            break;
        }
        n_alive = na2;
        uint32_t *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (done) {
        if (gtid == 0) {
            ctl->kappa = k;
            ctl->rounds = rounds;
            __hip_atomic_store(&ctl->qtail, tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    // Hand over to one workgroup.  Every remaining vertex is in cur with its degree (the number
    // of its remaining neighbours, since every queued vertex has been removed): give it a local
    // id and that many consecutive entries of the local adjacency (one 64-bit atomic per
    // wavefront reserves both, so rows follow local ids and lrow is a CSR row array), then write
    // its remaining neighbours' local ids there.
    for (uint32_t b0 = gwave * 64; b0 < n_alive; b0 += nwaves * 64) {
        const uint32_t i = b0 + lane;
        uint32_t v = 0;
        int d = -1;
        if (i < n_alive) {
            v = cur[i];
            d = ld_relaxed(&deg[v]);
        }
        const bool live = d >= 0;
        const uint64_t ml = __ballot(live);
        // inclusive prefix of the live degrees within the wavefront
        uint32_t inc = live ? (uint32_t)d : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= (unsigned)o) inc += y;
        }
        const uint32_t tot = __shfl(inc, 63, 64);
        unsigned long long base = 0;
        if (lane == 0 && ml)
            base = atomicAdd(&ctl->lres, ((unsigned long long)tot << 32) | (unsigned long long)__popcll(ml));
        base = __shfl(base, 0, 64);
        if (live) {
            const uint32_t lid = (uint32_t)base + (uint32_t)__popcll(ml & below);
            const uint64_t off = (base >> 32) + inc - (uint32_t)d;
            if (lid < kTail && off + (uint32_t)d <= lcol_cap) {
                rlist[lid] = v;
                loc[v] = lid;
                lrow[lid] = (uint32_t)off;
            } else {
                atomicOr(&ctl->error, 4u);
            }
        }
    }
    grid_barrier(ctl, btarget += nblk);
    const unsigned long long lres = __hip_atomic_load(&ctl->lres, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t R = (uint32_t)lres, total = (uint32_t)(lres >> 32);
    if (R != n - tail || R > kTail || total > lcol_cap || ld_relaxed(&ctl->error)) {
        if (gtid == 0) atomicOr(&ctl->error, 4u);
        return;
    }
    if (gtid == 0) {
        lrow[R] = total;
        ctl->ho_tail = tail;
        ctl->ho_k = k;
        ctl->ho_rounds = rounds;
        ctl->ho = 1;
    }
}

// The hand-over's local adjacency: for every local vertex, its remaining neighbours' local ids,
// found by a scan of its whole row with one wavefront.  A launch of its own on the whole device
// (the grid has narrowed by then, and the rows of the last vertices, hubs, are long).
__global__ void __launch_bounds__(256)
k_local_adj(const uint32_t *__restrict__ row, const uint32_t *__restrict__ col, const int *__restrict__ deg,
            const uint32_t *__restrict__ loc, const uint32_t *__restrict__ rlist, const uint32_t *__restrict__ lrow,
            uint16_t *__restrict__ lcol, PeelCtl *__restrict__ ctl) {
    if (!ctl->ho || ctl->error) return;
    const uint32_t R = (uint32_t)ctl->lres;
    const unsigned lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1;
    const uint32_t nwaves = gridDim.x * (256 / 64);
    for (uint32_t l = blockIdx.x * (256 / 64) + threadIdx.x / 64; l < R; l += nwaves) {
        const uint32_t v = rlist[l], b = lrow[l];
        const uint32_t d = (uint32_t)deg[v];
        const uint32_t e = row[v + 1];
        uint32_t c = 0;
        for (uint32_t j0 = row[v]; j0 < e; j0 += 64) {
            const uint32_t j = j0 + lane;
            const uint32_t lx = j < e ? loc[col[j]] : kUnset;
            const uint64_t m = __ballot(lx != kUnset);
            const uint32_t p = c + (uint32_t)__popcll(m & below);
            if (lx != kUnset && p < d) lcol[b + p] = (uint16_t)lx;
            c += (uint32_t)__popcll(m);
        }
        if (lane == 0 && c != d) atomicOr(&ctl->error, 4u);
    }
}

// the one-workgroup finish after a hand-over
__global__ void __launch_bounds__(kBlock)
k_peel_finish(const uint32_t *__restrict__ rlist, const uint32_t *__restrict__ lrow, const uint16_t *__restrict__ lcol,
              uint32_t *__restrict__ lvl, uint32_t *__restrict__ level, uint32_t *__restrict__ queue,
              PeelCtl *__restrict__ ctl) {
    __shared__ __attribute__((aligned(16))) uint32_t s_mem[kLdsWords];
    if (!ctl->ho || ctl->error) return;
    peel_tail((uint32_t)ctl->lres, ctl->ho_tail, ctl->ho_k, ctl->ho_rounds, rlist, lrow, lcol, lvl, level, queue, ctl,
              s_mem);
}

__global__ void k_finish(uint32_t n, const uint32_t *__restrict__ queue, uint32_t *__restrict__ rank) {
    uint32_t p = blockIdx.x * 256 + threadIdx.x;
    if (p < n) rank[queue[p]] = p;
}

}  // namespace

int peel(dt_graph *g) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    DevMem deg, alive, alive2, ctlm, loc, rlist, lrow, lvl, lcol, ovf0, ovf1;
    DT_TRY(dev_alloc(ctx, deg, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, alive, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, alive2, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, ovf0, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, ovf1, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->core, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->order, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->rank, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, ctlm, sizeof(PeelCtl)));
    // the one-workgroup finish: at most tail_cap vertices, their adjacency within 2 m_static
    // entries and below tail_cap (tail_cap - 1) as well
    const uint32_t tail_cap = std::min<uint32_t>(g->tuning.peel_tail ? g->tuning.peel_tail : kTail, kTail);
    const uint64_t lcol_cap = std::min<uint64_t>(2ull * g->m_s, (uint64_t)tail_cap * (tail_cap - 1));
    DT_TRY(dev_alloc(ctx, loc, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, rlist, (uint64_t)tail_cap * 4));
    DT_TRY(dev_alloc(ctx, lrow, ((uint64_t)tail_cap + 1) * 4));
    DT_TRY(dev_alloc(ctx, lvl, (uint64_t)tail_cap * 8));
    DT_TRY(dev_alloc(ctx, lcol, (lcol_cap + 1) * 2));
    if (n == 0) {
        g->kappa = 0;
        g->peel_rounds = 0;
        return DT_OK;
    }
    // co-resident grid (the cooperative launch fails rather than run a grid that cannot be)
    int per_cu = 0;
    DT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_peel, kBlock, 0));
    if (per_cu <= 0) return fail(DT_EDEVICE, "peel kernel cannot be resident");
    unsigned grid = kGridWide;
    if (grid > (unsigned)ctx->num_cus * (unsigned)per_cu) grid = (unsigned)ctx->num_cus * (unsigned)per_cu;
    DT_HIP(hipMemsetAsync(ctlm.ptr, 0, sizeof(PeelCtl), st));
    uint32_t *level = g->core.as<uint32_t>();
    uint32_t *queue = g->order.as<uint32_t>();
    const uint32_t *row = g->row.as<uint32_t>(), *col = g->col.as<uint32_t>();
    int *degp = deg.as<int>();
    uint32_t *aa = alive.as<uint32_t>(), *ab = alive2.as<uint32_t>();
    PeelCtl *ctl = ctlm.as<PeelCtl>();
    uint32_t nn = n;
    uint32_t *locp = loc.as<uint32_t>(), *rl = rlist.as<uint32_t>(), *lb = lrow.as<uint32_t>(),
             *ld = lvl.as<uint32_t>();
    uint16_t *lc = lcol.as<uint16_t>();
    uint64_t lcap = lcol_cap;
    uint32_t tcap = tail_cap;
    uint32_t *o0 = ovf0.as<uint32_t>(), *o1 = ovf1.as<uint32_t>();
    void *args[] = {&nn, &row, &col, &degp, &level, &queue, &aa, &ab, &locp, &rl, &lb, &ld, &lc, &lcap, &tcap,
                    &o0, &o1, &ctl};
    prof_begin(ctx, kProfPeel, st);
    DT_HIP(hipLaunchCooperativeKernel((const void *)k_peel, dim3(grid), dim3(kBlock), args, 0, st));
    prof_end(ctx, kProfPeel, st);
    prof_begin(ctx, kProfPeelAdj, st);
    k_local_adj<<<(unsigned)ctx->num_cus * 8, 256, 0, st>>>(row, col, degp, locp, rl, lb, lc, ctl);
    prof_end(ctx, kProfPeelAdj, st);
    DT_HIP(hipGetLastError());
    prof_begin(ctx, kProfPeelTail, st);
    k_peel_finish<<<1, kBlock, 0, st>>>(rl, lb, lc, ld, level, queue, ctl);
    prof_end(ctx, kProfPeelTail, st);
    DT_HIP(hipGetLastError());
    PeelCtl h{};
    DT_HIP(hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    if (h.error & 1u) return fail(DT_EDEVICE, "core peel barrier timed out");
    if (h.error) return fail(DT_EDEVICE, "core peel failed its consistency checks (code %u)", h.error);
    if (h.qtail != n) return fail(DT_EDEVICE, "core peel queued %u of %u vertices", h.qtail, n);
    g->kappa = h.kappa;
    g->peel_rounds = h.rounds;
    g->alg_bytes_peel = 16ull * n + 16ull * g->m_s;
    // the ranks (what the orientation reads next, on the same stream); the temporaries released on
    // return were last used by kernels the read-back above waited for
    k_finish<<<grid_for(n, 256), 256, 0, st>>>(n, queue, g->rank.as<uint32_t>());
    DT_HIP(hipGetLastError());
    return DT_OK;
}

}  // namespace dt
