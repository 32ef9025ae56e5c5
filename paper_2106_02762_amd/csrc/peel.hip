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
// Small frontiers, which are most rounds on power-law graphs, are drained by one workgroup that
// loops over rounds on the device; a frontier above kSmallLimit goes back to the host, which
// launches a grid-wide round.
#include "internal.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;
constexpr unsigned kSmallBlock = 1024;
constexpr uint32_t kSmallLimit = 4096;
constexpr uint32_t kUnset = 0xffffffffu;

// device counters of the peel
struct PeelState {
    unsigned int qtail;      // vertices queued so far (positions in the ordering)
    unsigned int qhead;      // vertices whose neighbours have been processed
    unsigned int n_alive2;   // survivors of the last level scan
    unsigned int min_deg;    // smallest degree among survivors of the last scan
    unsigned int rounds;     // removal rounds done on the device
    unsigned int pad[3];
};

__global__ void k_init(uint32_t n, const uint32_t *__restrict__ row, int *__restrict__ deg,
                       uint32_t *__restrict__ level, uint32_t *__restrict__ alive) {
    uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    deg[v] = (int)(row[v + 1] - row[v]);
    level[v] = kUnset;
    alive[v] = v;
}

// Queue every remaining vertex of degree <= k; keep the others (and their smallest degree).
__global__ void k_level_scan(uint32_t n_alive, const uint32_t *__restrict__ alive, uint32_t k,
                             const int *__restrict__ deg, uint32_t *__restrict__ level,
                             uint32_t *__restrict__ queue, uint32_t *__restrict__ alive2,
                             PeelState *__restrict__ st) {
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_alive) return;
    uint32_t v = alive[i];
    if (level[v] != kUnset) return;
    int d = deg[v];
    if (d <= (int)k) {
        level[v] = k;
        uint32_t p = atomicAdd(&st->qtail, 1u);
        queue[p] = v;
    } else {
        uint32_t p = atomicAdd(&st->n_alive2, 1u);
        alive2[p] = v;
        atomicMin(&st->min_deg, (unsigned)d);
    }
}

// Remove queue[head..tail): one wavefront per vertex, lanes over its neighbours.
__device__ inline void remove_vertex(uint32_t v, uint32_t k, const uint32_t *__restrict__ row,
                                     const uint32_t *__restrict__ col, int *__restrict__ deg,
                                     uint32_t *__restrict__ level, uint32_t *__restrict__ queue,
                                     PeelState *__restrict__ st, unsigned lane) {
    uint32_t b = row[v], e = row[v + 1];
    for (uint32_t j = b + lane; j < e; j += 64) {
        uint32_t x = col[j];
        if (level[x] != kUnset) continue;
        int old = atomicSub(&deg[x], 1);
        if (old == (int)k + 1) {
            level[x] = k;
            uint32_t p = atomicAdd(&st->qtail, 1u);
            queue[p] = x;
        }
    }
}

__global__ void k_round(uint32_t head, uint32_t tail, uint32_t k, const uint32_t *__restrict__ row,
                        const uint32_t *__restrict__ col, int *__restrict__ deg,
                        uint32_t *__restrict__ level, uint32_t *__restrict__ queue,
                        PeelState *__restrict__ st) {
    uint32_t w = (blockIdx.x * kBlock + threadIdx.x) / 64;
    unsigned lane = threadIdx.x & 63;
    if (head + w >= tail) return;
    remove_vertex(queue[head + w], k, row, col, deg, level, queue, st, lane);
}

// One workgroup drains the level's queue round by round while the frontier stays small.
__global__ void __launch_bounds__(kSmallBlock)
k_drain_small(uint32_t k, const uint32_t *__restrict__ row, const uint32_t *__restrict__ col,
              int *__restrict__ deg, uint32_t *__restrict__ level, uint32_t *__restrict__ queue,
              PeelState *__restrict__ st) {
    __shared__ uint32_t s_head, s_tail;
    const unsigned wave = threadIdx.x / 64, lane = threadIdx.x & 63;
    constexpr unsigned kWaves = kSmallBlock / 64;
    for (;;) {
        if (threadIdx.x == 0) {
            s_head = atomicAdd(&st->qhead, 0u);
            s_tail = atomicAdd(&st->qtail, 0u);
        }
        __syncthreads();
        const uint32_t h = s_head, t = s_tail;
        __syncthreads();
        if (h == t || t - h > kSmallLimit) break;   // level done, or too big for one workgroup
        for (uint32_t i = h + wave; i < t; i += kWaves)
            remove_vertex(queue[i], k, row, col, deg, level, queue, st, lane);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            atomicExch(&st->qhead, t);
            atomicAdd(&st->rounds, 1u);
        }
        __syncthreads();
    }
}

__global__ void k_finish(uint32_t n, const uint32_t *__restrict__ queue, uint32_t *__restrict__ rank) {
    uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p < n) rank[queue[p]] = p;
}

}  // namespace

int peel(dt_graph *g) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    DevMem deg, alive, alive2, stm;
    DT_TRY(dev_alloc(ctx, deg, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, alive, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, alive2, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->core, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->order, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, g->rank, (uint64_t)n * 4));
    DT_TRY(dev_alloc(ctx, stm, sizeof(PeelState)));
    PeelState *dst = stm.as<PeelState>();
    uint32_t *level = g->core.as<uint32_t>();
    uint32_t *queue = g->order.as<uint32_t>();
    const uint32_t *row = g->row.as<uint32_t>(), *col = g->col.as<uint32_t>();
    if (n == 0) { g->kappa = 0; g->peel_rounds = 0; return DT_OK; }

    k_init<<<grid_for(n, kBlock), kBlock, 0, st>>>(n, row, deg.as<int>(), level, alive.as<uint32_t>());
    DT_HIP(hipGetLastError());
    PeelState h{};
    DT_HIP(hipMemcpyAsync(dst, &h, sizeof(h), hipMemcpyHostToDevice, st));

    uint32_t k = 0, n_alive = n, kappa = 0, host_rounds = 0, prev_tail = 0;
    uint32_t *a_cur = alive.as<uint32_t>(), *a_next = alive2.as<uint32_t>();
    while (true) {
        // reset the scan outputs, then scan the remaining vertices at level k
        unsigned int reset[2] = {0u, 0xffffffffu};
        DT_HIP(hipMemcpyAsync(&dst->n_alive2, reset, sizeof(reset), hipMemcpyHostToDevice, st));
        k_level_scan<<<grid_for(n_alive, kBlock), kBlock, 0, st>>>(n_alive, a_cur, k, deg.as<int>(),
                                                                   level, queue, a_next, dst);
        DT_HIP(hipGetLastError());
        k_drain_small<<<1, kSmallBlock, 0, st>>>(k, row, col, deg.as<int>(), level, queue, dst);
        DT_HIP(hipGetLastError());
        DT_HIP(hipMemcpyAsync(&h, dst, sizeof(h), hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
        // large frontiers: grid-wide rounds until the small drain can finish the level
        while (h.qhead != h.qtail) {
            uint32_t head = h.qhead, tail = h.qtail;
            uint64_t threads = (uint64_t)(tail - head) * 64;
            k_round<<<grid_for(threads, kBlock), kBlock, 0, st>>>(head, tail, k, row, col,
                                                                  deg.as<int>(), level, queue, dst);
            DT_HIP(hipGetLastError());
            host_rounds++;
            DT_HIP(hipMemcpyAsync(&dst->qhead, &tail, 4, hipMemcpyHostToDevice, st));
            k_drain_small<<<1, kSmallBlock, 0, st>>>(k, row, col, deg.as<int>(), level, queue, dst);
            DT_HIP(hipGetLastError());
            DT_HIP(hipMemcpyAsync(&h, dst, sizeof(h), hipMemcpyDeviceToHost, st));
            DT_HIP(hipStreamSynchronize(st));
        }
        if (h.qtail >= n) { if (h.qtail > 0) kappa = k; break; }
        // survivors of this level's scan that were not queued by its rounds stay for later levels
        n_alive = h.n_alive2;
        std::swap(a_cur, a_next);
        if (h.n_alive2 == 0) break;   // cannot happen with qtail < n, kept as a guard
        // every survivor now has degree > k; when this level removed nothing, no degree changed
        // since the scan, so the smallest survivor degree is the next level that removes anything
        uint32_t next = k + 1;
        if (h.qtail == prev_tail && h.min_deg != 0xffffffffu && h.min_deg > next) next = h.min_deg;
        prev_tail = h.qtail;
        k = next;
        if (k > n) return fail(DT_EDEVICE, "core peel did not terminate (k=%u)", k);
    }
    g->kappa = kappa;
    g->peel_rounds = h.rounds + host_rounds;
    k_finish<<<grid_for(n, kBlock), kBlock, 0, st>>>(n, queue, g->rank.as<uint32_t>());
    DT_HIP(hipGetLastError());
    DT_HIP(hipStreamSynchronize(st));
    return DT_OK;
}

}  // namespace dt
