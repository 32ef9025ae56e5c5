// Loading a temporal graph: the static graph G and the per-pair, per-direction edge store
// (Section 3 defines G and the multiplicities; Section 4 assumes constant-time access to each
// pair's edges in each direction in time order, which this CSR store provides).
//
// Every kept edge gets the 64-bit key ((t - t_min) << shift) | input_index, so that one unsigned
// comparison orders edges by (t, input index) and a time bound "t < x" is the key bound
// (x - t_min) << shift.
#include "internal.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;

__device__ inline uint64_t order_key(int64_t t) {   // int64 -> uint64, order preserving
    return (uint64_t)t ^ 0x8000000000000000ull;
}

__global__ void k_scan_input(uint32_t n, uint64_t m, const uint32_t *__restrict__ src,
                             const uint32_t *__restrict__ dst, const int64_t *__restrict__ t,
                             unsigned long long *__restrict__ out /* [0] bad ids, [1] self loops,
                                                                    [2] min key, [3] max key */) {
    __shared__ unsigned long long s_min[kBlock], s_max[kBlock], s_bad[kBlock], s_self[kBlock];
    unsigned long long mn = ~0ull, mx = 0, bad = 0, self = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * kBlock) {
        uint32_t a = src[i], b = dst[i];
        if (a >= n || b >= n) { bad++; continue; }
        if (a == b) { self++; continue; }
        uint64_t k = order_key(t[i]);
        mn = k < mn ? k : mn;
        mx = k > mx ? k : mx;
    }
    s_min[threadIdx.x] = mn; s_max[threadIdx.x] = mx; s_bad[threadIdx.x] = bad; s_self[threadIdx.x] = self;
    __syncthreads();
    for (unsigned w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            unsigned o = threadIdx.x + w;
            s_min[threadIdx.x] = s_min[o] < s_min[threadIdx.x] ? s_min[o] : s_min[threadIdx.x];
            s_max[threadIdx.x] = s_max[o] > s_max[threadIdx.x] ? s_max[o] : s_max[threadIdx.x];
            s_bad[threadIdx.x] += s_bad[o];
            s_self[threadIdx.x] += s_self[o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (s_bad[0]) atomicAdd(&out[0], s_bad[0]);
        if (s_self[0]) atomicAdd(&out[1], s_self[0]);
        atomicMin(&out[2], s_min[0]);
        atomicMax(&out[3], s_max[0]);
    }
}

// time key of every input edge; self-loops get ~0 so that they sort last
__global__ void k_time_keys(uint64_t m, const uint32_t *__restrict__ src,
                            const uint32_t *__restrict__ dst, const int64_t *__restrict__ t,
                            int64_t t_min, int shift, uint64_t *__restrict__ key,
                            uint32_t *__restrict__ idx) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    key[i] = src[i] == dst[i] ? ~0ull : ((uint64_t)(t[i] - t_min) << shift) | i;
    idx[i] = (uint32_t)i;
}

// unordered pair key (x << 32 | y, x < y) of each kept edge in time order
__global__ void k_pair_keys(uint64_t m, const uint32_t *__restrict__ idx_t,
                            const uint32_t *__restrict__ src, const uint32_t *__restrict__ dst,
                            uint64_t *__restrict__ pk, uint32_t *__restrict__ j_out) {
    uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= m) return;
    uint32_t i = idx_t[j];
    uint32_t a = src[i], b = dst[i];
    uint32_t x = a < b ? a : b, y = a < b ? b : a;
    pk[j] = ((uint64_t)x << 32) | y;
    j_out[j] = (uint32_t)j;
}

__global__ void k_run_heads(uint64_t m, const uint64_t *__restrict__ pk, uint32_t *__restrict__ head) {
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m) return;
    head[k] = (k == 0 || pk[k] != pk[k - 1]) ? 1u : 0u;
}

// per kept edge in pair order: pair id, key, direction; per pair: endpoints and first edge
__global__ void k_fill_pairs(uint64_t m, const uint64_t *__restrict__ pk, const uint32_t *__restrict__ jv,
                             const uint32_t *__restrict__ head, const uint32_t *__restrict__ excl,
                             const uint64_t *__restrict__ tkey, const uint32_t *__restrict__ idx_t,
                             const uint32_t *__restrict__ src, const uint32_t *__restrict__ dst,
                             uint32_t *__restrict__ psid, uint64_t *__restrict__ pkey,
                             uint8_t *__restrict__ pdir, uint32_t *__restrict__ sx,
                             uint32_t *__restrict__ sy, uint32_t *__restrict__ pstart) {
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m) return;
    uint32_t s = excl[k] + head[k] - 1;
    psid[k] = s;
    uint64_t p = pk[k];
    if (head[k]) {
        sx[s] = (uint32_t)(p >> 32);
        sy[s] = (uint32_t)p;
        pstart[s] = (uint32_t)k;
    }
    uint32_t j = jv[k];
    pkey[k] = tkey[j];
    uint32_t i = idx_t[j];
    pdir[k] = src[i] > dst[i] ? 1 : 0;
}

__global__ void k_dir_flags(uint64_t m, const uint8_t *__restrict__ pdir, uint32_t *__restrict__ f) {
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < m) f[k] = pdir[k];
}

__global__ void k_max_mult(uint64_t ms, uint64_t m, const uint32_t *__restrict__ pstart,
                           unsigned int *__restrict__ out) {
    __shared__ unsigned s_max[kBlock];
    unsigned mx = 0;
    for (uint64_t s = (uint64_t)blockIdx.x * kBlock + threadIdx.x; s < ms;
         s += (uint64_t)gridDim.x * kBlock) {
        uint64_t e = s + 1 < ms ? pstart[s + 1] : m;
        unsigned c = (unsigned)(e - pstart[s]);
        mx = c > mx ? c : mx;
    }
    s_max[threadIdx.x] = mx;
    __syncthreads();
    for (unsigned w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s_max[threadIdx.x] = max(s_max[threadIdx.x], s_max[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, s_max[0]);
}

__global__ void k_adj_keys(uint64_t ms, const uint32_t *__restrict__ sx, const uint32_t *__restrict__ sy,
                           uint64_t *__restrict__ ak, uint32_t *__restrict__ av,
                           uint32_t *__restrict__ deg) {
    uint64_t s = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= ms) return;
    uint32_t x = sx[s], y = sy[s];
    ak[2 * s] = ((uint64_t)x << 32) | y;
    ak[2 * s + 1] = ((uint64_t)y << 32) | x;
    av[2 * s] = (uint32_t)s;
    av[2 * s + 1] = (uint32_t)s;
    atomicAdd(&deg[x], 1u);
    atomicAdd(&deg[y], 1u);
}

__global__ void k_low_words(uint64_t n, const uint64_t *__restrict__ k, uint32_t *__restrict__ lo) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) lo[i] = (uint32_t)k[i];
}

int bits_for(uint64_t x) {   // smallest b >= 1 with x <= 2^b
    int b = 1;
    while (b < 64 && (1ull << b) < x) b++;
    return b;
}

}  // namespace

int load_graph(dt_graph *g, const uint32_t *src, const uint32_t *dst, const int64_t *t) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint64_t m_in = g->m_in;
    const uint32_t n = g->n;

    // 1. validate ids, count self-loops, time range
    DevMem scal;
    DT_TRY(dev_alloc(ctx, scal, 8 * sizeof(unsigned long long)));
    unsigned long long h_init[4] = {0, 0, ~0ull, 0};
    DT_HIP(hipMemcpyAsync(scal.ptr, h_init, sizeof(h_init), hipMemcpyHostToDevice, st));
    if (m_in) {
        unsigned grid = grid_for(m_in, kBlock);
        if (grid > 4096) grid = 4096;
        k_scan_input<<<grid, kBlock, 0, st>>>(n, m_in, src, dst, t, scal.as<unsigned long long>());
        DT_HIP(hipGetLastError());
    }
    unsigned long long h[4];
    DT_HIP(hipMemcpyAsync(h, scal.ptr, sizeof(h), hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    if (h[0]) return fail(DT_EINVAL, "%llu edges name a vertex id >= n = %u", h[0], n);
    g->self_loops = h[1];
    g->m = m_in - h[1];
    const uint64_t m = g->m;
    if (m) {
        g->t_min = (int64_t)(h[2] ^ 0x8000000000000000ull);
        g->t_max = (int64_t)(h[3] ^ 0x8000000000000000ull);
    } else {
        g->t_min = g->t_max = 0;
    }
    g->span = g->t_max - g->t_min;
    g->shift = bits_for(m_in);
    if (m && ((uint64_t)g->span >> (64 - g->shift)) != 0)
        return fail(DT_EOVERFLOW, "time span %lld does not fit beside a %d-bit edge index",
                    (long long)g->span, g->shift);
    if (m && (uint64_t)g->span + 2 >= (1ull << (64 - g->shift)))
        return fail(DT_EOVERFLOW, "time span %lld too close to the %d-bit key limit",
                    (long long)g->span, 64 - g->shift);

    // 2. keys in (t, index) order
    DevMem tk, tidx, tk2, tidx2;
    DT_TRY(dev_alloc(ctx, tk, m_in * 8));
    DT_TRY(dev_alloc(ctx, tidx, m_in * 4));
    DT_TRY(dev_alloc(ctx, tk2, m_in * 8));
    DT_TRY(dev_alloc(ctx, tidx2, m_in * 4));
    if (m_in) {
        k_time_keys<<<grid_for(m_in, kBlock), kBlock, 0, st>>>(m_in, src, dst, t, g->t_min, g->shift,
                                                               tk.as<uint64_t>(), tidx.as<uint32_t>());
        DT_HIP(hipGetLastError());
        DT_TRY(sort_pairs_u64_u32(ctx, tk.as<uint64_t>(), tk2.as<uint64_t>(), tidx.as<uint32_t>(),
                                  tidx2.as<uint32_t>(), m_in, 64, st));
    }
    tk.reset();
    tidx.reset();

    // 3. group by unordered pair (stable, so each pair's edges stay in key order)
    DevMem pk, jv, pk2, jv2;
    DT_TRY(dev_alloc(ctx, pk, m * 8));
    DT_TRY(dev_alloc(ctx, jv, m * 4));
    DT_TRY(dev_alloc(ctx, pk2, m * 8));
    DT_TRY(dev_alloc(ctx, jv2, m * 4));
    const int pair_bits = 32 + bits_for((uint64_t)n + 1);
    if (m) {
        k_pair_keys<<<grid_for(m, kBlock), kBlock, 0, st>>>(m, tidx2.as<uint32_t>(), src, dst,
                                                            pk.as<uint64_t>(), jv.as<uint32_t>());
        DT_HIP(hipGetLastError());
        DT_TRY(sort_pairs_u64_u32(ctx, pk.as<uint64_t>(), pk2.as<uint64_t>(), jv.as<uint32_t>(),
                                  jv2.as<uint32_t>(), m, pair_bits, st));
    }
    pk.reset();
    jv.reset();

    // 4. pair ids, endpoints, per-edge key and direction
    DevMem head, excl;
    DT_TRY(dev_alloc(ctx, head, m * 4));
    DT_TRY(dev_alloc(ctx, excl, m * 4));
    uint64_t ms = 0;
    if (m) {
        k_run_heads<<<grid_for(m, kBlock), kBlock, 0, st>>>(m, pk2.as<uint64_t>(), head.as<uint32_t>());
        DT_HIP(hipGetLastError());
        DT_TRY(exclusive_scan_u32(ctx, head.as<uint32_t>(), excl.as<uint32_t>(), m, st));
        uint32_t last[2];
        DT_HIP(hipMemcpyAsync(&last[0], excl.as<uint32_t>() + (m - 1), 4, hipMemcpyDeviceToHost, st));
        DT_HIP(hipMemcpyAsync(&last[1], head.as<uint32_t>() + (m - 1), 4, hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
        ms = (uint64_t)last[0] + last[1];
    }
    g->m_s = ms;
    DT_TRY(dev_alloc(ctx, g->sx, ms * 4));
    DT_TRY(dev_alloc(ctx, g->sy, ms * 4));
    DT_TRY(dev_alloc(ctx, g->pstart, (ms + 1) * 4));
    DT_TRY(dev_alloc(ctx, g->psid, m * 4));
    DT_TRY(dev_alloc(ctx, g->pkey, m * 8));
    DT_TRY(dev_alloc(ctx, g->pdir, m));
    g->max_mult = 0;
    if (m) {
        k_fill_pairs<<<grid_for(m, kBlock), kBlock, 0, st>>>(
            m, pk2.as<uint64_t>(), jv2.as<uint32_t>(), head.as<uint32_t>(), excl.as<uint32_t>(),
            tk2.as<uint64_t>(), tidx2.as<uint32_t>(), src, dst, g->psid.as<uint32_t>(),
            g->pkey.as<uint64_t>(), g->pdir.as<uint8_t>(), g->sx.as<uint32_t>(), g->sy.as<uint32_t>(),
            g->pstart.as<uint32_t>());
        DT_HIP(hipGetLastError());
        uint32_t mm = (uint32_t)m;
        DT_HIP(hipMemcpyAsync(g->pstart.as<uint32_t>() + ms, &mm, 4, hipMemcpyHostToDevice, st));
        DT_HIP(hipMemsetAsync(scal.ptr, 0, 4, st));
        unsigned grid = grid_for(ms, kBlock);
        if (grid > 4096) grid = 4096;
        k_max_mult<<<grid, kBlock, 0, st>>>(ms, m, g->pstart.as<uint32_t>(), scal.as<unsigned>());
        DT_HIP(hipGetLastError());
        DT_HIP(hipMemcpyAsync(&g->max_mult, scal.ptr, 4, hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
    }
    pk2.reset(); jv2.reset(); head.reset(); excl.reset(); tk2.reset(); tidx2.reset();

    // count of head -> tail edges (pdir = 1) before every position, for the re-layout by direction
    {
        DevMem flag;
        DT_TRY(dev_alloc(ctx, flag, (m + 1) * 4));
        DT_TRY(dev_alloc(ctx, g->c1, (m + 1) * 4));
        DT_HIP(hipMemsetAsync(flag.ptr, 0, (m + 1) * 4, st));
        if (m) {
            k_dir_flags<<<grid_for(m, kBlock), kBlock, 0, st>>>(m, g->pdir.as<uint8_t>(), flag.as<uint32_t>());
            DT_HIP(hipGetLastError());
        }
        DT_TRY(exclusive_scan_u32(ctx, flag.as<uint32_t>(), g->c1.as<uint32_t>(), m + 1, st));
    }

    // 5. undirected CSR of G with pair ids, neighbours sorted by id
    DevMem ak, av, ak2, deg;
    DT_TRY(dev_alloc(ctx, ak, 2 * ms * 8));
    DT_TRY(dev_alloc(ctx, av, 2 * ms * 4));
    DT_TRY(dev_alloc(ctx, ak2, 2 * ms * 8));
    DT_TRY(dev_alloc(ctx, g->ceid, 2 * ms * 4));
    DT_TRY(dev_alloc(ctx, g->col, 2 * ms * 4));
    DT_TRY(dev_alloc(ctx, deg, ((uint64_t)n + 1) * 4));
    DT_TRY(dev_alloc(ctx, g->row, ((uint64_t)n + 1) * 4));
    DT_HIP(hipMemsetAsync(deg.ptr, 0, ((uint64_t)n + 1) * 4, st));
    if (ms) {
        k_adj_keys<<<grid_for(ms, kBlock), kBlock, 0, st>>>(ms, g->sx.as<uint32_t>(), g->sy.as<uint32_t>(),
                                                            ak.as<uint64_t>(), av.as<uint32_t>(),
                                                            deg.as<uint32_t>());
        DT_HIP(hipGetLastError());
        DT_TRY(sort_pairs_u64_u32(ctx, ak.as<uint64_t>(), ak2.as<uint64_t>(), av.as<uint32_t>(),
                                  g->ceid.as<uint32_t>(), 2 * ms, pair_bits, st));
        k_low_words<<<grid_for(2 * ms, kBlock), kBlock, 0, st>>>(2 * ms, ak2.as<uint64_t>(),
                                                                 g->col.as<uint32_t>());
        DT_HIP(hipGetLastError());
    }
    DT_TRY(exclusive_scan_u32(ctx, deg.as<uint32_t>(), g->row.as<uint32_t>(), (uint64_t)n + 1, st));
    DT_HIP(hipStreamSynchronize(st));
    return DT_OK;
}

}  // namespace dt
