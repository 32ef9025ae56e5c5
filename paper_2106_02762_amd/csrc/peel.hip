// Degeneracy ordering by a parallel k-core peel (Section 3: "removing a vertex with minimum degree
// repeatedly"; the degeneracy is the largest core number).
//
// Level k removes every remaining vertex whose remaining degree is <= k, in rounds: the vertices
// found by a scan of the remaining ones, then those whose degree falls to k while their
// neighbours are removed.  A vertex's position in the ordering is the order in which it joined the
// removal queue.  When v joins, at most k of its neighbours are still unqueued, and every
// neighbour that comes after v in the ordering is one of them, so the out-degree of v in G_prec
// is at most k = core(v) <= degeneracy, the property Theorem 1's bound rests on.  (Different
// removal orders give different orientations but the same counts: each static triangle is
// counted once under its own naming u < v < w.)
//
// The whole peel is one cooperative (co-resident) grid of a few blocks: levels and rounds are
// separated by grid barriers instead of kernel launches and host round trips, since power-law
// graphs need thousands of rounds, most with frontiers of a few vertices.  A barrier's cost grows
// with the number of blocks that meet at it, so the grid is small and wide (32 blocks of 1024
// threads), and the barrier is a counter whose last arriving block also snapshots the queue and
// survivor counters before it releases the others: each round then needs one barrier, and every
// block takes the same branch because all decisions use the snapshot.  A vertex is queued at most
// once: by the level scan when its degree is <= k (no decrement runs during a scan), or by the
// single decrement that takes its degree from k + 1 to k (degrees only fall, and a queued vertex
// already has degree <= k, so no later decrement can see k + 1 again); the queue index is also
// bounds-checked, and the host checks that exactly n vertices were queued.  A barrier that waits far longer than any peel could take sets an error
// flag and lets its block go, so that a fault in this logic ends the kernel instead of hanging it.
#include "internal.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 1024;
constexpr unsigned kGridBlocks = 32;
constexpr uint32_t kUnset = 0xffffffffu;
constexpr long kSpinLimit = 1l << 26;

struct PeelCtl {
    unsigned int qtail;      // vertices queued so far (positions in the ordering)
    unsigned int n_alive2;   // survivors of the current level scan
    unsigned int min_deg;    // smallest degree among those survivors
    unsigned int arrived;    // barrier arrivals
    unsigned int gen;        // barrier generation
    unsigned int error;      // a barrier gave up waiting
    unsigned int rounds;     // removal rounds
    unsigned int kappa;      // largest level that removed a vertex
    unsigned int snap[2][4]; // per generation parity: qtail, n_alive2, min_deg at the release
};

__device__ __forceinline__ unsigned ld_relaxed(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier; returns the snapshot taken by the last block to arrive.  With reset_scan the
// survivor counters are cleared after the snapshot, ready for the next level scan.
__device__ void grid_barrier(PeelCtl *ctl, unsigned nblk, bool reset_scan, unsigned snap[3]) {
    __shared__ unsigned s_gen;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned my = __hip_atomic_load(&ctl->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned arrived = atomicAdd(&ctl->arrived, 1u) + 1;
        if (arrived == nblk) {
            const unsigned par = my & 1u;
            ctl->snap[par][0] = ld_relaxed(&ctl->qtail);
            ctl->snap[par][1] = ld_relaxed(&ctl->n_alive2);
            ctl->snap[par][2] = ld_relaxed(&ctl->min_deg);
            if (reset_scan) {
                __hip_atomic_store(&ctl->n_alive2, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctl->min_deg, 0xffffffffu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __hip_atomic_store(&ctl->arrived, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&ctl->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spins = 0;
            while (__hip_atomic_load(&ctl->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == my) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kSpinLimit) {
                    atomicOr(&ctl->error, 1u);
                    break;
                }
            }
        }
        s_gen = my;
    }
    __syncthreads();
    const unsigned par = s_gen & 1u;
    snap[0] = ld_relaxed(&ctl->snap[par][0]);
    snap[1] = ld_relaxed(&ctl->snap[par][1]);
    snap[2] = ld_relaxed(&ctl->snap[par][2]);
}

__device__ __forceinline__ void enqueue(uint32_t v, uint32_t k, uint32_t n, uint32_t *level,
                                        uint32_t *queue, PeelCtl *ctl) {
    level[v] = k;
    uint32_t p = atomicAdd(&ctl->qtail, 1u);
    if (p < n) queue[p] = v;
}

__device__ __forceinline__ void remove_edges(uint32_t v, uint32_t first, uint32_t stride, uint32_t k,
                                             uint32_t n, const uint32_t *__restrict__ row,
                                             const uint32_t *__restrict__ col, int *__restrict__ deg,
                                             uint32_t *__restrict__ level, uint32_t *__restrict__ queue,
                                             PeelCtl *ctl) {
    const uint32_t e = row[v + 1];
    for (uint32_t j = row[v] + first; j < e; j += stride) {
        const uint32_t x = col[j];
        const int old = atomicSub(&deg[x], 1);
        if (old == (int)k + 1) enqueue(x, k, n, level, queue, ctl);
    }
}

__global__ void __launch_bounds__(kBlock)
k_peel(uint32_t n, const uint32_t *__restrict__ row, const uint32_t *__restrict__ col,
       int *__restrict__ deg, uint32_t *__restrict__ level, uint32_t *__restrict__ queue,
       uint32_t *__restrict__ alive_a, uint32_t *__restrict__ alive_b, PeelCtl *__restrict__ ctl) {
    const unsigned nblk = gridDim.x;
    const uint32_t gtid = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t gsize = nblk * kBlock;
    const uint32_t gwave = gtid / 64, nwaves = gsize / 64, lane = threadIdx.x & 63;
    unsigned snap[3];

    // the host cleared the control block; initialise per-vertex state
    for (uint32_t v = gtid; v < n; v += gsize) {
        deg[v] = (int)(row[v + 1] - row[v]);
        level[v] = kUnset;
        alive_a[v] = v;
    }
    grid_barrier(ctl, nblk, true, snap);

    uint32_t k = 0, head = 0, n_alive = n, prev_tail = 0, rounds = 0;
    uint32_t *cur = alive_a, *nxt = alive_b;
    while (true) {
        // level scan: queue every remaining vertex of degree <= k, keep the others
        for (uint32_t i = gtid; i < n_alive; i += gsize) {
            const uint32_t v = cur[i];
            if (ld_relaxed(&level[v]) != kUnset) continue;
            const int d = ld_relaxed(&deg[v]);
            if (d <= (int)k) {
                enqueue(v, k, n, level, queue, ctl);
            } else {
                nxt[atomicAdd(&ctl->n_alive2, 1u)] = v;
                atomicMin(&ctl->min_deg, (unsigned)d);
            }
        }
        grid_barrier(ctl, nblk, true, snap);
        uint32_t tail = snap[0];
        const uint32_t na2 = snap[1], md = snap[2];
        // rounds: remove queue[head, tail).  A frontier of at least one vertex per wavefront is
        // split by vertex; a smaller one gives each vertex an equal share of the wavefronts.
        while (head < tail) {
            const uint32_t f = tail - head;
            if (f >= nwaves) {
                for (uint32_t i = head + gwave; i < tail; i += nwaves)
                    remove_edges(queue[i], lane, 64, k, n, row, col, deg, level, queue, ctl);
            } else {
                const uint32_t per = nwaves / f;
                const uint32_t i = gwave / per, sub = gwave % per;
                if (i < f)
                    remove_edges(queue[head + i], sub * 64 + lane, per * 64, k, n, row, col, deg,
                                 level, queue, ctl);
            }
            ++rounds;
            grid_barrier(ctl, nblk, false, snap);
            head = tail;
            tail = snap[0];
        }
        if (tail >= n || ld_relaxed(&ctl->error)) break;
        // every survivor now has degree > k; when this level removed nothing, no degree changed
        // since the scan, so the smallest survivor degree is the next level that removes anything
        uint32_t next = k + 1;
        if (tail == prev_tail && md != 0xffffffffu && md > next) next = md;
        prev_tail = tail;
        k = next;
        if (k > n + 1) {   // cannot happen: some vertex is removed at the smallest survivor degree
            if (gtid == 0) atomicOr(&ctl->error, 2u);
            break;
        }
        n_alive = na2;
        uint32_t *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (gtid == 0) {
        ctl->kappa = k;
        ctl->rounds = rounds;
    }
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
    DevMem deg, alive, alive2, ctlm;
    DT_TRY(dev_alloc(ctx, deg, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, alive, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, alive2, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->core, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->order, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->rank, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, ctlm, sizeof(PeelCtl)));
    if (n == 0) {
        g->kappa = 0;
        g->peel_rounds = 0;
        return DT_OK;
    }
    // co-resident grid (the cooperative launch fails rather than run a grid that cannot be)
    int per_cu = 0;
    DT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_peel, kBlock, 0));
    if (per_cu <= 0) return fail(DT_EDEVICE, "peel kernel cannot be resident");
    unsigned grid = kGridBlocks;
    if (grid > (unsigned)ctx->num_cus * (unsigned)per_cu) grid = (unsigned)ctx->num_cus * (unsigned)per_cu;
    DT_HIP(hipMemsetAsync(ctlm.ptr, 0, sizeof(PeelCtl), st));
    uint32_t *level = g->core.as<uint32_t>();
    uint32_t *queue = g->order.as<uint32_t>();
    const uint32_t *row = g->row.as<uint32_t>(), *col = g->col.as<uint32_t>();
    int *degp = deg.as<int>();
    uint32_t *aa = alive.as<uint32_t>(), *ab = alive2.as<uint32_t>();
    PeelCtl *ctl = ctlm.as<PeelCtl>();
    uint32_t nn = n;
    void *args[] = {&nn, &row, &col, &degp, &level, &queue, &aa, &ab, &ctl};
    prof_begin(ctx, kProfPeel, st);
    DT_HIP(hipLaunchCooperativeKernel((const void *)k_peel, dim3(grid), dim3(kBlock), args, 0, st));
    prof_end(ctx, kProfPeel, st);
    PeelCtl h{};
    DT_HIP(hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    if (h.error) return fail(DT_EDEVICE, "core peel barrier timed out");
    if (h.qtail != n) return fail(DT_EDEVICE, "core peel queued %u of %u vertices", h.qtail, n);
    g->kappa = h.kappa;
    g->peel_rounds = h.rounds;
    g->alg_bytes_peel = 16ull * n + 16ull * g->m_s;
    k_finish<<<grid_for(n, 256), 256, 0, st>>>(n, queue, g->rank.as<uint32_t>());
    DT_HIP(hipGetLastError());
    DT_HIP(hipStreamSynchronize(st));
    return DT_OK;
}

}  // namespace dt
