// Orientation of G by the degeneracy ordering into the DAG G_prec (Section 3: orient {u, v} from
// u to v iff u comes first), and the re-layout of the temporal edge store in DAG-edge order.
//
// Vertices are renamed by their rank, so a DAG edge is (rank u, rank v) with rank u < rank v and
// the out-neighbours of u are a sorted run.  The runs are built without a global sort: out-degrees
// are counted from the pair list, scanned into rows, every pair is placed in its tail's run, and
// each run (at most the degeneracy long) is sorted by one wavefront.  DAG edges are numbered in
// (tail, head) order, and the
// temporal edges of DAG edge d are stored at [eoff[2d], eoff[2d+2]): first those directed
// tail -> head, then head -> tail, each in key order (a scatter by rank, no re-sort).  The
// enumeration of triangles reads only the offsets, so a build moves the keys on a side stream
// while it runs.  All edges at one source vertex u are then
// one contiguous stretch of the store, which is exactly what the counting of all triangles with
// source u walks (Section 5: only {u,v} and {u,w} are enumerated).
#include "internal.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;

// Lanes with equal keys in consecutive lanes form runs; the first lane of a run adds the run's
// length to ctr[key] with one atomic, and each lane gets the old value plus its offset in the run.
__device__ __forceinline__ uint32_t run_add(uint32_t *ctr, uint32_t key, bool active, unsigned lane) {
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool prev_active = __shfl_up(active ? 1 : 0, 1, 64) != 0;
    const bool head = active && (lane == 0 || !prev_active || prev != key);
    const uint64_t heads = __ballot(head), acts = __ballot(active);
    const uint64_t upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1);
    const uint64_t mine = heads & upto;
    const unsigned start = mine ? 63 - __clzll(mine) : 0;
    // the run ends at the next head or inactive lane
    const uint64_t stops = (heads | ~acts) & ~upto;
    const unsigned end = stops ? (unsigned)__ffsll((unsigned long long)stops) - 1 : 64;
    uint32_t old = 0;
    if (head) old = atomicAdd(&ctr[key], end - start);
    old = __shfl(old, start, 64);
    return old + (lane - start);
}

// out-degree of every rank (each static pair points from its lower-ranked end), and per pair its
// (tail, head) ranks and whether the DAG direction swaps the pair's (sx -> sy) direction
__global__ void k_dag_count(uint64_t ms, const uint32_t *__restrict__ sx, const uint32_t *__restrict__ sy,
                            const uint32_t *__restrict__ rank, uint32_t *__restrict__ outdeg,
                            uint2 *__restrict__ th, uint8_t *__restrict__ sflip) {
    const uint64_t s = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool act = s < ms;
    uint32_t tail = 0;
    if (act) {
        const uint32_t ra = rank[sx[s]], rb = rank[sy[s]];
        tail = ra < rb ? ra : rb;
        th[s] = make_uint2(tail, ra < rb ? rb : ra);
        sflip[s] = ra < rb ? 0 : 1;
    }
    (void)run_add(outdeg, tail, act, threadIdx.x & 63);
}

// every pair into its tail's run (unordered) as (head rank, pair id, edges tail -> head,
// edges head -> tail)
__global__ void k_dag_place(uint64_t ms, const uint2 *__restrict__ th, const uint8_t *__restrict__ sflip,
                            const uint32_t *__restrict__ pstart, const uint32_t *__restrict__ c1,
                            const uint32_t *__restrict__ dag_row, uint32_t *__restrict__ cursor,
                            uint4 *__restrict__ runs) {
    const uint64_t s = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool act = s < ms;
    uint2 e = make_uint2(0, 0);
    if (act) e = th[s];
    const uint32_t off = run_add(cursor, e.x, act, threadIdx.x & 63);
    if (act) {
        const uint32_t ps = pstart[s], pe = pstart[s + 1];
        const uint32_t n1 = c1[pe] - c1[ps], n0 = (pe - ps) - n1;   // pdir 1: sy -> sx
        const bool flip = sflip[s] != 0;
        runs[dag_row[e.x] + off] = make_uint4(e.y, (uint32_t)s, flip ? n1 : n0, flip ? n0 : n1);
    }
}

// DAG edge d: its head, its pair's DAG id, and the sizes of its two direction groups
__device__ __forceinline__ void dag_edge(uint64_t d, uint4 r, uint32_t *__restrict__ dag_col,
                                         uint32_t *__restrict__ dag_of, uint32_t *__restrict__ gsize) {
    dag_col[d] = r.x;
    dag_of[r.y] = (uint32_t)d;
    gsize[2 * d] = r.z;
    gsize[2 * d + 1] = r.w;
}

// Sort every run by head rank (heads are distinct).  Wavefronts take chunks of kTailChunk tails
// from a work counter; runs that fit together in 64 lanes are loaded in one piece and sorted at
// once: each entry placed at the number of (run, head) keys below its own, or, past 2^26
// vertices, by a bitonic network on (run, head).  Longer runs are left to k_dag_sort_long.
constexpr uint32_t kTailChunk = 64;

__global__ void __launch_bounds__(kBlock)
k_dag_sort(uint32_t n, const uint32_t *__restrict__ dag_row, const uint4 *__restrict__ runs,
           uint32_t *__restrict__ dag_col, uint32_t *__restrict__ dag_of, uint32_t *__restrict__ gsize,
           unsigned *__restrict__ next_chunk) {
    const unsigned lane = threadIdx.x & 63;
    for (;;) {
        uint32_t t0 = 0;
        if (lane == 0) t0 = atomicAdd(next_chunk, kTailChunk);
        t0 = __shfl(t0, 0, 64);
        if (t0 >= n) break;
        const uint32_t t1 = t0 + kTailChunk < n ? t0 + kTailChunk : n;
        uint32_t r = t0;
        while (r < t1) {
            const uint32_t b = dag_row[r];
            // lane l: end of run r + l (relative to b) if that tail is in the chunk
            const uint32_t endl = r + lane < t1 ? dag_row[r + lane + 1] - b : 0xffffffffu;
            const uint64_t fits = __ballot(endl <= 64);
            const uint32_t cnt = fits == ~0ull ? 64u : (uint32_t)__ffsll((unsigned long long)~fits) - 1;
            if (cnt == 0) {   // run r alone exceeds 64: listed by k_long_runs, sorted by k_dag_sort_long
                r += 1;
                continue;
            }
            const uint32_t len = __shfl(endl, cnt - 1, 64);
            // run of lane x: the number of runs ending at or before x
            uint32_t seg = 0;
            for (uint32_t q = 0; q < cnt; ++q) seg += __shfl(endl, q, 64) <= lane ? 1u : 0u;
            uint4 rec = make_uint4(0xffffffffu, 0, 0, 0);
            uint64_t key = ~0ull;
            if (lane < len) {
                rec = runs[b + lane];
                key = ((uint64_t)seg << 32) | rec.x;
            }
            if (n <= (1u << 26)) {
                // (run, head) fits 32 bits and is distinct per lane: each entry's place is the number
                // of lanes with a smaller one
                const uint32_t k32 = lane < len ? (seg << 26) | rec.x : 0xffffffffu;
                uint32_t pos = 0;
                for (uint32_t q = 0; q < len; ++q) pos += __shfl(k32, q, 64) < k32 ? 1u : 0u;
                if (lane < len) dag_edge(b + pos, rec, dag_col, dag_of, gsize);
                r += cnt;
                continue;
            }
#pragma unroll
            for (unsigned k = 2; k <= 64; k <<= 1) {
#pragma unroll
                for (unsigned j = k >> 1; j > 0; j >>= 1) {
                    const uint64_t ok = __shfl_xor(key, j, 64);
                    const uint32_t o0 = __shfl_xor(rec.x, j, 64), o1 = __shfl_xor(rec.y, j, 64),
                                   o2 = __shfl_xor(rec.z, j, 64), o3 = __shfl_xor(rec.w, j, 64);
                    const bool take_min = ((lane & j) == 0) == ((lane & k) == 0);
                    const bool other = take_min ? ok < key : key < ok;
                    if (other) {
                        key = ok;
                        rec = make_uint4(o0, o1, o2, o3);
                    }
                }
            }
            if (lane < len) dag_edge(b + lane, rec, dag_col, dag_of, gsize);
            r += cnt;
        }
    }
}

// the tails whose runs are longer than 64 (one atomic per wavefront)
__global__ void k_long_runs(uint32_t n, const uint32_t *__restrict__ dag_row, unsigned *__restrict__ n_long,
                            uint32_t *__restrict__ longs) {
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    const unsigned lane = threadIdx.x & 63;
    const bool is_long = t < n && dag_row[t + 1] - dag_row[t] > 64;
    const uint64_t m = __ballot(is_long);
    if (!m) return;
    unsigned base = 0;
    if (lane == 0) base = atomicAdd(n_long, (unsigned)__popcll(m));
    base = __shfl(base, 0, 64);
    if (is_long) longs[base + (unsigned)__popcll(m & ((1ull << lane) - 1))] = t;
}

// Runs longer than 64: one workgroup per run.  Heads within a run are distinct, so an entry's place
// is the number of heads below its own: the run's heads are staged in LDS and every thread counts,
// for each of its entries (held in registers), the heads below it in one pass over them (each LDS
// read serves the whole wavefront; no barrier between compare steps).  Runs past kLongCap entries,
// beyond any degeneracy met in practice, are ranked the same way in global memory.
constexpr uint32_t kLongCap = 2048;
constexpr uint32_t kLongPer = kLongCap / kBlock;   // entries of a run per thread

// pos[e] += heads of sh[0, L) below rec[e].x, for the first M entries
template <int M>
__device__ __forceinline__ void count_below(const uint32_t *sh, uint32_t L, const uint4 (&rec)[kLongPer],
                                            uint32_t (&pos)[kLongPer]) {
    for (uint32_t j = 0; j < L; ++j) {
        const uint32_t hj = sh[j];
#pragma unroll
        for (int e = 0; e < M; ++e) pos[e] += hj < rec[e].x ? 1u : 0u;
    }
}

__global__ void __launch_bounds__(kBlock)
k_dag_sort_long(const unsigned *__restrict__ n_long_p, const uint32_t *__restrict__ longs,
                const uint32_t *__restrict__ dag_row, const uint4 *__restrict__ runs,
                uint32_t *__restrict__ dag_col, uint32_t *__restrict__ dag_of, uint32_t *__restrict__ gsize) {
    __shared__ uint32_t sh[kLongCap];
    const unsigned n_long = *n_long_p;
    for (unsigned li = blockIdx.x; li < n_long; li += gridDim.x) {
        const uint32_t r = longs[li];
        const uint32_t b = dag_row[r], L = dag_row[r + 1] - b;
        if (L <= kLongCap) {
            uint4 rec[kLongPer];
            uint32_t pos[kLongPer];
#pragma unroll
            for (uint32_t e = 0; e < kLongPer; ++e) {
                const uint32_t i = threadIdx.x + e * kBlock;
                rec[e] = i < L ? runs[b + i] : make_uint4(0, 0, 0, 0);
                if (i < L) sh[i] = rec[e].x;
                pos[e] = 0;
            }
            __syncthreads();
            const uint32_t mine = (L > threadIdx.x ? L - threadIdx.x + kBlock - 1 : 0) / kBlock;   // entries held
            switch ((L + kBlock - 1) / kBlock) {   // the most entries a thread holds (uniform)
                case 1: count_below<1>(sh, L, rec, pos); break;
                case 2: count_below<2>(sh, L, rec, pos); break;
                case 3: count_below<3>(sh, L, rec, pos); break;
                case 4: count_below<4>(sh, L, rec, pos); break;
                case 5: count_below<5>(sh, L, rec, pos); break;
                case 6: count_below<6>(sh, L, rec, pos); break;
                case 7: count_below<7>(sh, L, rec, pos); break;
                default: count_below<8>(sh, L, rec, pos); break;
            }
#pragma unroll
            for (uint32_t e = 0; e < kLongPer; ++e)
                if (e < mine) dag_edge(b + pos[e], rec[e], dag_col, dag_of, gsize);
            __syncthreads();
        } else {
            for (uint32_t i = threadIdx.x; i < L; i += kBlock) {
                const uint32_t h = runs[b + i].x;
                uint32_t pos = 0;
                for (uint32_t j = 0; j < L; ++j) pos += runs[b + j].x < h ? 1u : 0u;
                dag_edge(b + pos, runs[b + i], dag_col, dag_of, gsize);
            }
        }
    }
}

// largest out-degree: max of row[i + 1] - row[i] over i < n
__global__ void k_max_u32(uint64_t n, const uint32_t *__restrict__ row, unsigned *__restrict__ out) {
    __shared__ unsigned s[kBlock];
    unsigned mx = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) {
        const unsigned dg = row[i + 1] - row[i];
        mx = dg > mx ? dg : mx;
    }
    s[threadIdx.x] = mx;
    __syncthreads();
    for (unsigned w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, s[0]);
}

// Move every temporal edge (pair-major, key order within the pair) to its place in the DAG-edge
// layout: group 2d + direction, at its rank among the pair's edges of that direction.  Ranks come
// from the running count c1 of head->tail flags, so each group stays in key order.
__global__ void k_relayout(uint64_t m, const uint32_t *__restrict__ psid, const uint8_t *__restrict__ pdir,
                           const uint32_t *__restrict__ pstart, const uint32_t *__restrict__ c1,
                           const uint32_t *__restrict__ dag_of, const uint8_t *__restrict__ sflip,
                           const uint32_t *__restrict__ eoff, const uint64_t *__restrict__ pkey,
                           uint64_t *__restrict__ key) {
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m) return;
    const uint32_t s = psid[k], ps = pstart[s], dir = pdir[k];
    const uint32_t ones = c1[k] - c1[ps];
    const uint32_t r = dir ? ones : (uint32_t)(k - ps) - ones;
    const uint32_t g = 2 * dag_of[s] + (dir ^ sflip[s]);
    key[eoff[g] + r] = pkey[k];
}

}  // namespace

int relayout_join(dt_graph *g) {
    if (!g->relay_pending) return DT_OK;
    g->relay_pending = false;
    const hipError_t e = hipStreamWaitEvent(g->ctx->stream, g->ctx->ev_relay[1], 0);
    // released in stream order on the context's stream, now behind the re-layout
    for (DevMem &t : g->relay_tmp) t.reset();
    if (e != hipSuccess) return fail(DT_EDEVICE, "hipStreamWaitEvent failed: %s", hipGetErrorString(e));
    return DT_OK;
}

int orient(dt_graph *g, bool overlap) {
    DT_TRY(relayout_join(g));   // (a build joins its own re-layout before returning)
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint64_t ms = g->m_s, m = g->m;
    const uint32_t n = g->n;
    DevMem outdeg, cursor, th, runs, longs, dag_of, sflip, gsize, scal;
    const uint64_t ngroups = 2 * ms;
    DT_TRY(dev_alloc(ctx, outdeg, ((uint64_t)n + 1) * 4));
    DT_TRY(dev_alloc(ctx, cursor, ((uint64_t)n + 1) * 4));
    DT_TRY(dev_alloc(ctx, th, ms * 8));
    DT_TRY(dev_alloc(ctx, runs, ms * 16));
    DT_TRY(dev_alloc(ctx, longs, ((uint64_t)n + 1) * 4));
    DT_TRY(dev_alloc(ctx, dag_of, ms * 4));
    DT_TRY(dev_alloc(ctx, sflip, ms));
    DT_TRY(dev_alloc(ctx, gsize, (ngroups + 1) * 4));
    DT_TRY(dev_alloc(ctx, g->dag_col, ms * 4));
    DT_TRY(dev_alloc(ctx, g->dag_row, ((uint64_t)n + 1) * 4));
    DT_TRY(dev_alloc(ctx, g->eoff, (ngroups + 1) * 4));
    DT_TRY(dev_alloc(ctx, g->key, m * 8));
    DT_TRY(dev_alloc(ctx, scal, 256));
    DT_HIP(hipMemsetAsync(outdeg.ptr, 0, ((uint64_t)n + 1) * 4, st));
    DT_HIP(hipMemsetAsync(cursor.ptr, 0, ((uint64_t)n + 1) * 4, st));
    DT_HIP(hipMemsetAsync(gsize.ptr, 0, (ngroups + 1) * 4, st));
    DT_HIP(hipMemsetAsync(scal.ptr, 0, 256, st));
    if (ms) {
        k_dag_count<<<grid_for(ms, kBlock), kBlock, 0, st>>>(ms, g->sx.as<uint32_t>(), g->sy.as<uint32_t>(),
            g->rank.as<uint32_t>(), outdeg.as<uint32_t>(), th.as<uint2>(), sflip.as<uint8_t>());
        DT_HIP(hipGetLastError());
    }
    DT_TRY(exclusive_scan_u32(ctx, outdeg.as<uint32_t>(), g->dag_row.as<uint32_t>(), (uint64_t)n + 1, st));
    if (ms) {
        k_dag_place<<<grid_for(ms, kBlock), kBlock, 0, st>>>(ms, th.as<uint2>(), sflip.as<uint8_t>(),
            g->pstart.as<uint32_t>(), g->c1.as<uint32_t>(), g->dag_row.as<uint32_t>(), cursor.as<uint32_t>(),
            runs.as<uint4>());
        DT_HIP(hipGetLastError());
        // runs of at most 64 on this stream, the longer ones beside them on side[1] (the two write
        // disjoint DAG edges; every buffer they use lives until this function returns, after the join)
        k_long_runs<<<grid_for(n, kBlock), kBlock, 0, st>>>(n, g->dag_row.as<uint32_t>(), scal.as<unsigned>() + 16,
                                                            longs.as<uint32_t>());
        DT_HIP(hipGetLastError());
        hipStream_t ls = ctx->side[1] ? ctx->side[1] : st;
        if (ls != st) {
            DT_HIP(hipEventRecord(ctx->ev_relay[0], st));
            DT_HIP(hipStreamWaitEvent(ls, ctx->ev_relay[0], 0));
        }
        k_dag_sort_long<<<(unsigned)ctx->num_cus * 4, kBlock, 0, ls>>>(scal.as<unsigned>() + 16, longs.as<uint32_t>(),
            g->dag_row.as<uint32_t>(), runs.as<uint4>(), g->dag_col.as<uint32_t>(), dag_of.as<uint32_t>(),
            gsize.as<uint32_t>());
        DT_HIP(hipGetLastError());
        k_dag_sort<<<(unsigned)ctx->num_cus * 8, kBlock, 0, st>>>(n, g->dag_row.as<uint32_t>(), runs.as<uint4>(),
            g->dag_col.as<uint32_t>(), dag_of.as<uint32_t>(), gsize.as<uint32_t>(), scal.as<unsigned>() + 8);
        DT_HIP(hipGetLastError());
        if (ls != st) {
            DT_HIP(hipEventRecord(ctx->ev_relay[1], ls));
            DT_HIP(hipStreamWaitEvent(st, ctx->ev_relay[1], 0));
        }
    }
    if (n) {
        unsigned grid = grid_for(n, kBlock);
        if (grid > 2048) grid = 2048;
        k_max_u32<<<grid, kBlock, 0, st>>>(n, g->dag_row.as<uint32_t>(), scal.as<unsigned>());
        DT_HIP(hipGetLastError());
    }
    // with overlap the store offsets' scan and the re-layout go to side[0] and keep their inputs
    // and temporaries alive until relayout_join; nothing on the context's stream reads g->eoff or
    // g->key before that (the enumeration reads only the DAG)
    const hipStream_t rs = overlap && m && ctx->side[0] ? ctx->side[0] : st;
    if (rs != st) {
        DT_HIP(hipEventRecord(ctx->ev_relay[0], st));
        DT_HIP(hipStreamWaitEvent(rs, ctx->ev_relay[0], 0));
    }
    DevMem scan_tmp;
    DT_TRY(exclusive_scan_u32(ctx, gsize.as<uint32_t>(), g->eoff.as<uint32_t>(), ngroups + 1, rs,
                              rs != st ? &scan_tmp : nullptr));
    if (m) {
        prof_begin(ctx, kProfRelayout, rs);
        k_relayout<<<grid_for(m, kBlock), kBlock, 0, rs>>>(m, g->psid.as<uint32_t>(), g->pdir.as<uint8_t>(),
            g->pstart.as<uint32_t>(), g->c1.as<uint32_t>(), dag_of.as<uint32_t>(), sflip.as<uint8_t>(),
            g->eoff.as<uint32_t>(), g->pkey.as<uint64_t>(), g->key.as<uint64_t>());
        prof_end(ctx, kProfRelayout, rs);
        DT_HIP(hipGetLastError());
        if (rs != st) {
            DT_HIP(hipEventRecord(ctx->ev_relay[1], rs));
            g->relay_tmp[0] = std::move(dag_of);
            g->relay_tmp[1] = std::move(sflip);
            g->relay_tmp[2] = std::move(gsize);
            g->relay_tmp[3] = std::move(scan_tmp);
            g->relay_pending = true;
        }
    }
    unsigned mo = 0;
    DT_HIP(hipMemcpyAsync(&mo, scal.ptr, 4, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    g->max_outdeg = mo;
    return DT_OK;
}

}  // namespace dt
