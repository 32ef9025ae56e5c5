// Static triangle enumeration in G_prec (Section 5 and the proof of Theorem 1): for every DAG
// edge (u, v) and every w in N+(u), {u, v, w} is a triangle iff w is also in N+(v); u is then the
// source vertex and u < v < w in the ordering.  The paper tests {v, w} with a hash lookup; here
// one wavefront owns one source vertex u and stages N+(u) (at most degeneracy entries) in LDS.
// For each v in N+(u) the two sorted runs N+(u) after v and N+(v) are intersected by walking the
// shorter and binary-searching the longer (hub vertices late in the ordering have long N+(v)
// runs reached from many u).  The candidates of all v are spread over the 64 lanes through a
// prefix sum of those walk lengths; a hit yields the DAG edge ids of {u, w} and {v, w} directly.
// Searches into N+(v) (when it is the longer run) take a rank-window bitmap of N+(v) instead, when
// v has one: before the pass, every vertex whose N+(v) has at least kBmMin heads within a window
// of kBmWin ranks gets its heads as bits over that window, each 32-bit word stored with the number
// of heads before it, so a membership test and the head's position in N+(v) are one 8-byte load
// (a hub's bitmap is read by all its in-neighbours and stays in cache).  Without a bitmap, a long
// walk over N+(u) (kStage entries or more) copies N+(v) into LDS and searches it there, a short
// one searches N+(v) in global memory.
//
// Waves take source vertices from the highest rank down, so the heaviest (the dense core, last in
// the ordering) start first.  One pass writes the list: each wavefront buffers its triangles in
// LDS and appends them with one atomic per buffer, so triangles sharing a source vertex stay
// mostly adjacent (as do their edge lists in the temporal store); the list's order is otherwise
// unspecified.  The list is sized at four triangles per static pair and the pass runs again at
// the counted size when a graph has more.  A vertex whose N+(u) exceeds the LDS slice takes the
// same steps on global memory (degeneracy above the slice, as in the densest inputs of Table 1).
#include <algorithm>

#include "count_dev.h"

namespace dt {

namespace {

constexpr unsigned kBlock = 256;
constexpr unsigned kWaves = kBlock / 64;
constexpr uint32_t kCap = 512;    // LDS entries of N+(u) (and of one N+(v)) per wavefront
constexpr uint32_t kStage = 32;   // walks at least this long search an LDS copy of N+(v)
// Work grabs of one counter, heaviest (highest-ranked) source vertices first: the first kSplitU
// vertices are split into kParts tickets each (part p takes every kParts-th block of 64 flattened
// candidates and every kParts-th staged neighbour), the next kSingles are one ticket each, and
// later tickets are kChunk vertices each.  No wavefront serialises the dense core.
constexpr uint32_t kSplitU = 8192, kParts = 8;   // kSplitU 4096: +0.5 ms; 16384: +0.3 ms (61M-edge graph)
constexpr uint32_t kSingles = 16384;
constexpr uint32_t kChunk = 16;
constexpr uint32_t kOut = 192;    // triangles a wavefront buffers in LDS before appending them
// list positions a wavefront reserves at once (one atomic on the shared counter per kChunkTri
// triangles instead of one per buffer: thousands of wavefronts meeting at one counter serialise)
constexpr uint32_t kChunkTri = 2048;
static_assert(kChunkTri >= kOut, "a buffer fits a fresh chunk");
constexpr int kBatchBuild = 4;    // blocks of 64 flattened candidates a lane works on at once
constexpr int kBatchFused = 1;    // (one in the one-shot pass: its counting holds the registers)
constexpr uint32_t kBmMin = 16;      // heads of N+(v) at least for a bitmap
constexpr uint32_t kBmWin = 32768;   // ranks a bitmap spans at most (1024 words)
constexpr uint32_t kBmWords = kBmWin / 32;
constexpr uint64_t kBmBudgetSlots = 1ull << 28;   // bitmap words of one graph at most (2 GiB)

// Bitmap of N+(v): info = (first head, words, slot base low, slot base high); words = 0: none.
// Slot x holds (heads before word x) << 32 | word x.  Returns whether w is a head of v and its
// position in N+(v).
__device__ __forceinline__ bool bm_find(const uint4 info, const uint64_t *__restrict__ slots, uint32_t w,
                                        uint32_t &pos) {
    const uint32_t off = w - info.x;   // wraps when w precedes the window
    if (off >= info.y * 32u) return false;
    const uint64_t slot = slots[((uint64_t)info.w << 32 | info.z) + (off >> 5)];
    const uint32_t word = (uint32_t)slot, bit = off & 31u;
    pos = (uint32_t)(slot >> 32) + (uint32_t)__popc(word & ((1u << bit) - 1u));
    return (word >> bit) & 1u;
}

// words of the bitmap of every vertex (0: none)
__global__ void k_bm_sizes(uint32_t n, const uint32_t *__restrict__ dag_row, const uint32_t *__restrict__ dag_col,
                           uint64_t *__restrict__ words) {
    const uint32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const uint32_t vb = dag_row[v], outv = dag_row[v + 1] - vb;
    uint64_t nw = 0;
    if (outv >= kBmMin) {
        const uint32_t win = dag_col[vb + outv - 1] - dag_col[vb] + 1;
        if (win <= kBmWin) nw = (win + 31) / 32;
    }
    words[v] = nw;
}

// the info of every vertex (slot bases from the exclusive scan of the words; none when off)
__global__ void k_bm_info(uint32_t n, const uint32_t *__restrict__ dag_row, const uint32_t *__restrict__ dag_col,
                          const uint64_t *__restrict__ words, const uint64_t *__restrict__ base, int on,
                          uint4 *__restrict__ info) {
    const uint32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const uint32_t nw = on ? (uint32_t)words[v] : 0u;
    const uint64_t b = base[v];
    info[v] = make_uint4(nw ? dag_col[dag_row[v]] : 0u, nw, (uint32_t)b, (uint32_t)(b >> 32));
}

// the slots of every bitmap: one wavefront per vertex builds its words in LDS, then writes them 64
// at a time with the running count of heads before each (a wave scan per 64 words)
__global__ void __launch_bounds__(256)
k_bm_fill(uint32_t n, const uint32_t *__restrict__ dag_row, const uint32_t *__restrict__ dag_col,
          const uint4 *__restrict__ info, uint64_t *__restrict__ slots) {
    __shared__ uint32_t s_bm[4][kBmWords];
    const unsigned lane = threadIdx.x & 63, wave = threadIdx.x / 64;
    uint32_t *bm = s_bm[wave];
    const uint32_t nw_all = gridDim.x * 4;
    for (uint32_t v = blockIdx.x * 4 + wave; v < n; v += nw_all) {
        const uint4 in = info[v];
        const uint32_t nw = in.y;   // words of this bitmap (at most kBmWords)
        if (nw == 0) continue;
        const uint32_t vb = dag_row[v], outv = dag_row[v + 1] - vb;
        for (uint32_t x = lane; x < nw; x += 64) bm[x] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        for (uint32_t j = lane; j < outv; j += 64) {
            const uint32_t off = dag_col[vb + j] - in.x;
            atomicOr(&bm[off >> 5], 1u << (off & 31));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        const uint64_t base = (uint64_t)in.w << 32 | in.z;
        uint32_t carry = 0;
        for (uint32_t w0 = 0; w0 < nw; w0 += 64) {
            const uint32_t wx = w0 + lane;
            const uint32_t word = wx < nw ? bm[wx] : 0u;
            const uint32_t c = (uint32_t)__popc(word);
            uint32_t incl = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o, 64);
                if (lane >= (unsigned)o) incl += y;
            }
            if (wx < nw) slots[base + wx] = (uint64_t)(carry + incl - c) << 32 | word;
            carry += __shfl(incl, 63, 64);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

__device__ __forceinline__ uint32_t find_u32(const uint32_t *a, uint32_t lo, uint32_t hi, uint32_t x) {
    uint32_t len = hi - lo;
    while (len > 0) {
        uint32_t half = len >> 1;
        if (a[lo + half] < x) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

// position i with pre[i] <= p < pre[i + 1] (pre ascending, pre[0] = 0, du entries)
__device__ __forceinline__ uint32_t owner(const uint32_t *pre, uint32_t du, uint32_t p) {
    uint32_t lo = 0, len = du;
    while (len > 0) {
        uint32_t half = len >> 1;
        if (pre[lo + half] <= p) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo - 1;
}

// What the one-shot (fused) pass needs to count triangles as it finds them.
struct FusedArgs {
    const uint32_t *eoff;
    const uint64_t *key;
    DQuery q;
    cdev::UQuery u;
    uint32_t unit_ok;              // unit records are exact (time span below 2^31)
    uint64_t cap_l;                // light rule: P <= cap_l and at most kLightVw {v,w} edges
    int shift;
    uint32_t *rest;                // other triangles, three DAG edge ids each
    uint64_t rest_cap;
    unsigned long long *rest_n;
    int64_t *part;                 // int64[8] per wavefront of the grid
    unsigned long long *s3;        // sum of sigma_uv sigma_uw sigma_vw, 128 bits (low, high)
};

// Buffered output: a wavefront collects its triangles in LDS and copies each full buffer into a
// stretch of list positions it reserved with one atomic per kChunkTri positions; when the stretch
// lacks room for a buffer, its rest is filled with empty triangles (all three ids kNoEdge) and a new
// stretch is taken, and at the end the unused rest of the last one is filled the same way.  The
// list therefore holds every triangle once and some empty entries, which the schedule skips; the
// wavefronts also add up the triangles they found.  Positions past `cap` are counted but not
// written.  In the one-shot
// pass (FUSED) a full buffer is counted instead: each lane takes every 64th buffered triangle;
// one with a single temporal edge per pair is tested as a unit record, a light one is counted
// pairwise in the lane, and the others go to the rest list for the medium and heavy paths (one
// atomic per wavefront and step); the wavefront's triangle count is added once, at the end.
template <bool FUSED>
struct TriSink {
    uint32_t *buf;      // LDS, 3 * kOut words
    uint32_t n;         // triangles buffered
    uint32_t *tri;
    uint64_t cap;
    unsigned long long *total;
    const FusedArgs *fa;
    unsigned long long *found_total;   // triangles found (stored pass)
    unsigned long long found = 0;   // triangles this wavefront found (counted, in the one-shot pass)
    unsigned long long cb = 0, ce = 0;   // the reserved positions [cb, ce) not yet used (stored pass)
    bool chunked = true;                 // stretches of kChunkTri positions, else one per buffer
    int64_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long s3lo = 0, s3hi = 0;
    // counts one triangle; false when it belongs to the medium or heavy paths (the rest list)
    __device__ __forceinline__ bool count_one(uint32_t a, uint32_t b, uint32_t c) {
        const FusedArgs &F = *fa;
        const uint32_t *eoff = F.eoff;
        const uint64_t s_uv = eoff[2 * a + 2] - eoff[2 * a], s_uw = eoff[2 * b + 2] - eoff[2 * b],
                       s_vw = eoff[2 * c + 2] - eoff[2 * c];
        const unsigned __int128 p3 = (unsigned __int128)(s_uv * s_uw) * s_vw;
        const unsigned long long lo = (unsigned long long)p3;
        s3lo += lo;
        s3hi += (unsigned long long)(p3 >> 64) + (s3lo < lo ? 1ull : 0ull);
        if (F.unit_ok && s_uv == 1 && s_uw == 1 && s_vw == 1) {
            uint32_t cc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            cdev::unit_one<false>(cdev::unit_record(a, b, c, eoff, F.key, F.shift), F.u, cc, nullptr);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] += cc[j];
        } else if (s_uv * s_uw <= F.cap_l && s_vw <= cdev::kLightVw) {
            cdev::Acc<false> A;
            cdev::Lists L;
            cdev::load_lists(eoff, a, b, c, F.key, F.q, L);
            cdev::light_pairs<0, 0>(F.key, L, F.q, A);
            cdev::light_pairs<0, 1>(F.key, L, F.q, A);
            cdev::light_pairs<1, 0>(F.key, L, F.q, A);
            cdev::light_pairs<1, 1>(F.key, L, F.q, A);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] += A.t[j];
        } else {
            return false;
        }
        return true;
    }

    __device__ __forceinline__ void flush(unsigned lane) {
        if (n == 0) return;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (FUSED) {
            found += n;
            // each lane counts every 64th buffered triangle; the rest list takes one atomic per step
            const FusedArgs &F = *fa;
            for (uint32_t x0 = 0; x0 < n; x0 += 64) {
                const uint32_t x = x0 + lane;
                uint32_t a = 0, b = 0, c = 0;
                bool rest = false;
                if (x < n) {
                    a = buf[3 * x];
                    b = buf[3 * x + 1];
                    c = buf[3 * x + 2];
                    rest = !count_one(a, b, c);
                }
                const uint64_t m = __ballot(rest);
                if (!m) continue;
                unsigned long long r0 = 0;
                if (lane == 0) r0 = atomicAdd(F.rest_n, (unsigned long long)__popcll(m));
                r0 = __shfl(r0, 0, 64);
                if (rest) {
                    const unsigned long long r = r0 + (unsigned long long)__popcll(m & ((1ull << lane) - 1));
                    if (r < F.rest_cap) {
                        F.rest[3 * r] = a;
                        F.rest[3 * r + 1] = b;
                        F.rest[3 * r + 2] = c;
                    }
                }
            }
        } else {
            found += n;
            if (ce - cb < n) {
                // a new stretch: kChunkTri positions, or exactly this buffer's (chunked = false)
                fill_empty(lane);
                const unsigned long long want = chunked ? kChunkTri : n;
                unsigned long long b = 0;
                if (lane == 0) b = atomicAdd(total, want);
                b = __shfl(b, 0, 64);
                cb = b;
                ce = b + want;
            }
            const unsigned long long base = cb;
            cb += n;
            for (uint32_t x = lane; x < 3 * n; x += 64)
                if (base + x / 3 < cap) tri[3 * base + x] = buf[x];
        }
        __builtin_amdgcn_wave_barrier();
        n = 0;
    }

    // the reserved positions [cb, ce) become empty triangles
    __device__ __forceinline__ void fill_empty(unsigned lane) {
        for (unsigned long long q = cb + lane; q < ce; q += 64)
            if (q < cap) {
                tri[3 * q] = kNoEdge;
                tri[3 * q + 1] = kNoEdge;
                tri[3 * q + 2] = kNoEdge;
            }
        cb = ce;
    }

    // at the end: the buffer out, the rest of the stretch emptied, and the wavefront's triangles
    // added up (to the found counter, or in the one-shot pass to the total)
    __device__ __forceinline__ void finish(unsigned lane) {
        flush(lane);
        if (FUSED) {
            if (lane == 0 && found) atomicAdd(total, found);
        } else {
            fill_empty(lane);
            if (lane == 0 && found) atomicAdd(found_total, found);
        }
    }

    // the lanes with hit set hold one triangle each; mask = the wave's ballot of hit
    __device__ __forceinline__ void put(bool hit, uint64_t mask, unsigned lane, uint32_t a, uint32_t b,
                                        uint32_t c) {
        const uint32_t nh = (uint32_t)__popcll(mask);
        if (nh == 0) return;
        if (n + nh > kOut) flush(lane);
        if (hit) {
            const uint32_t r = n + (uint32_t)__popcll(mask & ((1ull << lane) - 1));
            buf[3 * r] = a;
            buf[3 * r + 1] = b;
            buf[3 * r + 2] = c;
        }
        n += nh;
    }
};

template <bool FUSED>
__global__ void __launch_bounds__(kBlock, 4)   // four wavefronts per SIMD (the LDS allows four blocks per CU)
k_tri(uint32_t n, const uint32_t *__restrict__ dag_row, const uint32_t *__restrict__ dag_col,
      uint32_t *__restrict__ tri, uint64_t cap, unsigned long long *__restrict__ total,
      unsigned int *__restrict__ next_u, unsigned long long *__restrict__ cand, FusedArgs fa,
      const uint4 *__restrict__ binfo, const uint64_t *__restrict__ bslots,
      unsigned long long *__restrict__ found_total, int chunked) {
    // per wavefront: N+(u), the run starts and (16-bit) lengths of each N+(v), and one slice that
    // holds the prefix of walk lengths during the flattened walks and then a staged N+(v) copy
    __shared__ uint32_t s_nbr[kWaves][kCap];
    __shared__ uint32_t s_pre[kWaves][kCap + 1];
    __shared__ uint32_t s_vb[kWaves][kCap];
    __shared__ uint16_t s_dv[kWaves][kCap];
    __shared__ uint32_t s_out[kWaves][3 * kOut];
    const unsigned wave = threadIdx.x / 64, lane = threadIdx.x & 63;
    uint32_t *nbr_lds = s_nbr[wave], *pre_lds = s_pre[wave], *vb_lds = s_vb[wave], *vn_lds = s_pre[wave];
    uint16_t *dv_lds = s_dv[wave];
    TriSink<FUSED> out{s_out[wave], 0, tri, cap, total, &fa, found_total};
    out.chunked = chunked != 0;
    unsigned long long wave_cand = 0;   // candidates tested, added once per wave
    for (;;) {
        uint32_t ticket = 0;
        if (lane == 0) ticket = atomicAdd(next_u, 1u);
        ticket = __shfl(ticket, 0, 64);
        uint64_t b64;
        uint32_t span, part = 0, parts = 1;
        if (ticket < kSplitU * kParts) {
            b64 = ticket / kParts;
            part = ticket % kParts;
            parts = kParts;
            span = 1;
        } else if (ticket < kSplitU * kParts + kSingles) {
            b64 = kSplitU + (ticket - kSplitU * kParts);
            span = 1;
        } else {
            b64 = kSplitU + kSingles + (uint64_t)(ticket - kSplitU * kParts - kSingles) * kChunk;
            span = kChunk;
        }
        if (b64 >= n) break;
        const uint32_t base = (uint32_t)b64;
        const uint32_t last = base + span < n ? base + span : n;
        // highest rank first: the dense core, with the longest N+ runs, comes last in the ordering
        for (uint32_t ci = base; ci < last; ++ci) {
        const uint32_t u = n - 1 - ci;
        const uint32_t r0 = dag_row[u], du = dag_row[u + 1] - r0;
        if (du < 2) continue;
        const bool in_lds = du <= kCap;
        const uint32_t *nbr = in_lds ? nbr_lds : dag_col + r0;
        // stage N+(u), the run start and length of each N+(v), and the prefix of the walk lengths
        // min(du - i - 1, d+(v)) (walks that search an LDS copy of N+(v) are taken later)
        uint32_t carry = 0;
        for (uint32_t b = 0; b < du; b += 64) {
            const uint32_t i = b + lane;
            uint32_t dv = 0;
            if (i < du) {
                const uint32_t v = dag_col[r0 + i];
                const uint32_t vb = dag_row[v], outv = dag_row[v + 1] - vb;
                const uint32_t after = du - i - 1;
                if (in_lds) {
                    nbr_lds[i] = v;
                    vb_lds[i] = vb;
                    dv_lds[i] = (uint16_t)(outv < 0xffffu ? outv : 0xffffu);
                }
                const bool staged = outv > after && after >= kStage && outv <= kCap;
                dv = in_lds ? (staged ? 0 : (outv < after ? outv : after)) : (i + 1 < du ? outv : 0);
            }
            uint32_t x = dv;   // inclusive wave scan
#pragma unroll
            for (int s = 1; s < 64; s <<= 1) {
                uint32_t y = __shfl_up(x, s, 64);
                if (lane >= (unsigned)s) x += y;
            }
            if (in_lds && i < du) pre_lds[i] = carry + x - dv;
            carry += __shfl(x, 63, 64);
        }
        const uint32_t work = carry;
        if (part == 0) wave_cand += work;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (in_lds) {
            // kBatch blocks of 64 candidates per step: their owners, then all their first loads,
            // then their searches in lockstep, so that kBatch global loads per lane are in flight
            // instead of one
            constexpr int kBatch = FUSED ? kBatchFused : kBatchBuild;
            for (uint32_t b = part * 64; b < work; b += parts * 64 * kBatch) {
                uint32_t ci[kBatch], cj[kBatch], cvb[kBatch], cov[kBatch], w[kBatch], lo[kBatch], len[kBatch];
                bool ok[kBatch], walk_v[kBatch];
#pragma unroll
                for (int x = 0; x < kBatch; ++x) {
                    const uint32_t p = b + (uint32_t)x * parts * 64 + lane;
                    ok[x] = p < work;
                    ci[x] = ok[x] ? owner(pre_lds, du, p) : 0u;
                    cj[x] = p - pre_lds[ci[x]];
                    cvb[x] = vb_lds[ci[x]];
                    const uint32_t d16 = dv_lds[ci[x]];
                    cov[x] = d16 != 0xffffu ? d16 : (ok[x] ? dag_row[nbr_lds[ci[x]] + 1] - cvb[x] : 0u);
                    // walk N+(v) and search N+(u) after v in LDS, or walk N+(u) after v and search
                    // N+(v) in global memory
                    walk_v[x] = cov[x] <= du - ci[x] - 1;
                }
#pragma unroll
                for (int x = 0; x < kBatch; ++x)
                    w[x] = !ok[x] ? 0u : (walk_v[x] ? dag_col[cvb[x] + cj[x]] : nbr_lds[ci[x] + 1 + cj[x]]);
                // searches in LDS (lower bound of w in nbr_lds[i + 1, du))
#pragma unroll
                for (int x = 0; x < kBatch; ++x) {
                    lo[x] = ci[x] + 1;
                    len[x] = ok[x] && walk_v[x] ? du - ci[x] - 1 : 0u;
                }
                while (true) {
                    bool more = false;
#pragma unroll
                    for (int x = 0; x < kBatch; ++x) {
                        if (!len[x]) continue;
                        const uint32_t half = len[x] >> 1;
                        if (nbr_lds[lo[x] + half] < w[x]) {
                            lo[x] += half + 1;
                            len[x] -= half + 1;
                        } else {
                            len[x] = half;
                        }
                        more |= len[x] != 0;
                    }
                    if (!more) break;
                }
                uint32_t pos[kBatch], bpos[kBatch];
                bool bhit[kBatch], bmap[kBatch];
#pragma unroll
                for (int x = 0; x < kBatch; ++x) {
                    pos[x] = lo[x];
                    lo[x] = cvb[x];
                    // N+(v) with a bitmap: one lookup instead of the search
                    bmap[x] = false;
                    bhit[x] = false;
                    bpos[x] = 0;
                    if (ok[x] && !walk_v[x]) {
                        const uint4 bi = binfo[nbr_lds[ci[x]]];
                        if (bi.y) {
                            bmap[x] = true;
                            bhit[x] = bm_find(bi, bslots, w[x], bpos[x]);
                        }
                    }
                    len[x] = ok[x] && !walk_v[x] && !bmap[x] ? cov[x] : 0u;
                }
                // searches in global memory (lower bound of w in N+(v)), loads of all kBatch together
                while (true) {
                    uint32_t val[kBatch];
#pragma unroll
                    for (int x = 0; x < kBatch; ++x) val[x] = len[x] ? dag_col[lo[x] + (len[x] >> 1)] : 0u;
                    bool more = false;
#pragma unroll
                    for (int x = 0; x < kBatch; ++x) {
                        if (!len[x]) continue;
                        const uint32_t half = len[x] >> 1;
                        if (val[x] < w[x]) {
                            lo[x] += half + 1;
                            len[x] -= half + 1;
                        } else {
                            len[x] = half;
                        }
                        more |= len[x] != 0;
                    }
                    if (!more) break;
                }
                uint32_t at[kBatch];
#pragma unroll
                for (int x = 0; x < kBatch; ++x) {
                    if (!ok[x]) at[x] = ~w[x];
                    else if (walk_v[x]) at[x] = pos[x] < du ? nbr_lds[pos[x]] : ~w[x];
                    else if (bmap[x]) at[x] = bhit[x] ? w[x] : ~w[x];
                    else at[x] = lo[x] < cvb[x] + cov[x] ? dag_col[lo[x]] : ~w[x];
                }
#pragma unroll
                for (int x = 0; x < kBatch; ++x) {
                    const bool hit = ok[x] && at[x] == w[x];
                    const uint32_t e_uw = walk_v[x] ? r0 + pos[x] : r0 + ci[x] + 1 + cj[x];
                    const uint32_t e_vw = walk_v[x] ? cvb[x] + cj[x] : (bmap[x] ? cvb[x] + bpos[x] : lo[x]);
                    out.put(hit, __ballot(hit), lane, r0 + ci[x], e_uw, e_vw);
                }
            }
            // long walks into a long N+(v): 64 positions of N+(u) are tested at once and the
            // bitmap infos of those taken here loaded together; then each in turn searches its
            // N+(v) by bitmap lookups or on an LDS copy
            for (uint32_t i0 = part; i0 + kStage < du; i0 += parts * 64) {
                const uint32_t il = i0 + lane * parts;
                bool take = false;
                uint4 bil = make_uint4(0, 0, 0, 0);
                if (il + kStage < du) {
                    const uint32_t after = du - il - 1, outv = dv_lds[il];   // 0xffff: longer than any stage
                    take = outv > after && after >= kStage && outv <= kCap;
                    if (take) bil = binfo[nbr_lds[il]];
                }
                for (uint64_t m = __ballot(take); m; m &= m - 1) {
                    const int src = __ffsll((unsigned long long)m) - 1;
                    const uint32_t i = i0 + (uint32_t)src * parts;
                    const uint32_t after = du - i - 1, outv = dv_lds[i];
                    const uint32_t vb = vb_lds[i];
                    wave_cand += after;
                    const uint4 bi = make_uint4(__shfl(bil.x, src, 64), __shfl(bil.y, src, 64), __shfl(bil.z, src, 64),
                                                __shfl(bil.w, src, 64));
                    if (bi.y) {
                        // N+(v) has a bitmap: one lookup per head of N+(u) after v
                        for (uint32_t b = 0; b < after; b += 64) {
                            const uint32_t j = b + lane;
                            bool hit = false;
                            uint32_t pos = 0;
                            if (j < after) hit = bm_find(bi, bslots, nbr_lds[i + 1 + j], pos);
                            out.put(hit, __ballot(hit), lane, r0 + i, r0 + i + 1 + j, vb + pos);
                        }
                        continue;
                    }
                    __builtin_amdgcn_wave_barrier();
                    for (uint32_t j = lane; j < outv; j += 64) vn_lds[j] = dag_col[vb + j];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __builtin_amdgcn_wave_barrier();
                    for (uint32_t b = 0; b < after; b += 64) {
                        const uint32_t j = b + lane;
                        bool hit = false;
                        uint32_t pos = 0;
                        if (j < after) {
                            const uint32_t w = nbr_lds[i + 1 + j];
                            pos = find_u32(vn_lds, 0, outv, w);
                            hit = pos < outv && vn_lds[pos] == w;
                        }
                        out.put(hit, __ballot(hit), lane, r0 + i, r0 + i + 1 + j, vb + pos);
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
        } else {
            // N+(u) larger than the LDS slice: the same candidates, v by v, on global memory (the
            // parts of a split vertex take every parts-th v)
            for (uint32_t i = part; i + 1 < du; i += parts) {
                const uint32_t v = nbr[i];
                const uint32_t b0 = dag_row[v], dv = dag_row[v + 1] - b0;
                for (uint32_t b = 0; b < dv; b += 64) {
                    const uint32_t j = b + lane;
                    bool hit = false;
                    uint32_t pos = 0;
                    if (j < dv) {
                        const uint32_t w = dag_col[b0 + j];
                        pos = find_u32(nbr, i + 1, du, w);
                        hit = pos < du && nbr[pos] == w;
                    }
                    out.put(hit, __ballot(hit), lane, r0 + i, r0 + pos, b0 + j);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        }
    }
    out.finish(lane);
    if (lane == 0) atomicAdd(cand, wave_cand);
    if (FUSED) {
        // this wavefront's sums: its partial slot, and the 128-bit multiplicity sum with carry
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t v = cdev::wave_sum((long long)out.acc[j]);
            if (lane == 0) fa.part[8 * ((uint64_t)blockIdx.x * kWaves + wave) + j] = v;
        }
        unsigned long long lo = out.s3lo, hi = out.s3hi;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long lo2 = __shfl_xor(lo, o, 64), hi2 = __shfl_xor(hi, o, 64);
            const unsigned long long sum = lo + lo2;
            hi = hi + hi2 + (sum < lo ? 1ull : 0ull);
            lo = sum;
        }
        if (lane == 0) {
            const unsigned long long old = atomicAdd(&fa.s3[0], lo);
            atomicAdd(&fa.s3[1], hi + (old + lo < old ? 1ull : 0ull));
        }
    }
}

// The rank-window bitmaps of the oriented graph (info per vertex, slots); none when they would
// pass kBmBudgetSlots words.
int build_bitmaps(const dt_graph *g, DevMem &info, DevMem &slots) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    DevMem words, base;
    DT_TRY(dev_alloc(ctx, info, (uint64_t)n * sizeof(uint4) + 16));
    DT_TRY(dev_alloc(ctx, words, ((uint64_t)n + 1) * 8));
    DT_TRY(dev_alloc(ctx, base, ((uint64_t)n + 1) * 8));
    DT_HIP(hipMemsetAsync(words.ptr, 0, ((uint64_t)n + 1) * 8, st));
    k_bm_sizes<<<grid_for(n, 256), 256, 0, st>>>(n, g->dag_row.as<uint32_t>(), g->dag_col.as<uint32_t>(),
                                                 words.as<uint64_t>());
    DT_HIP(hipGetLastError());
    DT_TRY(exclusive_scan_u64(ctx, words.as<uint64_t>(), base.as<uint64_t>(), (uint64_t)n + 1, st));
    uint64_t *h = reinterpret_cast<uint64_t *>(ctx->pinned_stage);
    DT_HIP(hipMemcpyAsync(h, base.as<uint64_t>() + n, 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    const uint64_t total = h[0];
    const int on = total > 0 && total <= kBmBudgetSlots;
    k_bm_info<<<grid_for(n, 256), 256, 0, st>>>(n, g->dag_row.as<uint32_t>(), g->dag_col.as<uint32_t>(),
                                                words.as<uint64_t>(), base.as<uint64_t>(), on, info.as<uint4>());
    DT_HIP(hipGetLastError());
    DT_TRY(dev_alloc(ctx, slots, (on ? total : 0) * 8 + 8));
    if (on) {
        k_bm_fill<<<(unsigned)ctx->num_cus * 8, 256, 0, st>>>(n, g->dag_row.as<uint32_t>(), g->dag_col.as<uint32_t>(),
                                                              info.as<uint4>(), slots.as<uint64_t>());
        DT_HIP(hipGetLastError());
    }
    return DT_OK;
}

}  // namespace

int enumerate_triangles(const dt_graph *g, DevMem &tri, uint64_t *ntri_out, uint64_t *cand_out,
                        uint64_t *nlist_out) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    *ntri_out = 0;
    *cand_out = 0;
    *nlist_out = 0;
    if (n == 0) return DT_OK;
    DevMem ctr, binfo, bslots;
    DT_TRY(dev_alloc(ctx, ctr, 256));
    DT_TRY(build_bitmaps(g, binfo, bslots));
    // room for 4 triangles per static pair.  Wavefronts reserve stretches of kChunkTri positions
    // when that room is at least four times what the last stretches of all wavefronts can leave
    // empty, else exactly each buffer's positions (no empty entries).  A graph with more triangles
    // runs the pass again, with room for its triangles and, with stretches, the most empty entries
    // they can leave: below kOut per stretch taken (at most one per kChunkTri - kOut triangles, and
    // one more per wavefront) and a last stretch per wavefront.
    uint64_t cap = std::max<uint64_t>(4ull * g->m_s, 1ull << 16);
    const unsigned grid = (unsigned)ctx->num_cus * 8;
    const uint64_t waves = (uint64_t)grid * kWaves;
    const int chunked = cap >= 4 * waves * kChunkTri ? 1 : 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        DT_TRY(dev_alloc(ctx, tri, cap * 12));
        DT_HIP(hipMemsetAsync(ctr.ptr, 0, 40, st));
        unsigned long long *c64 = reinterpret_cast<unsigned long long *>(ctr.as<uint8_t>() + 8);
        prof_begin(ctx, kProfTriFill, st);
        k_tri<false><<<grid, kBlock, 0, st>>>(n, g->dag_row.as<uint32_t>(), g->dag_col.as<uint32_t>(),
                                              tri.as<uint32_t>(), cap, c64, ctr.as<unsigned>(), c64 + 1, FusedArgs{},
                                              binfo.as<uint4>(), bslots.as<uint64_t>(), c64 + 2, chunked);
        prof_end(ctx, kProfTriFill, st);
        DT_HIP(hipGetLastError());
        uint64_t *h = reinterpret_cast<uint64_t *>(ctx->pinned_stage);
        DT_HIP(hipMemcpyAsync(h, c64, 24, hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
        *nlist_out = h[0];
        *cand_out = h[1];
        *ntri_out = h[2];
        if (h[0] <= cap) return DT_OK;
        const uint64_t stretches = h[2] / (kChunkTri - kOut) + 2 * waves;
        cap = chunked ? h[2] + stretches * kOut + waves * kChunkTri : h[2];
        tri.reset();
    }
    return fail(DT_EDEVICE, "triangle enumeration changed between passes");
}

int fused_count(dt_graph *g, const DQuery &q, int64_t *out8_dev, DevMem &rest, uint64_t *n_rest, uint64_t *ntri_out,
                uint64_t *cand_out) {
    dt_ctx *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    *n_rest = *ntri_out = *cand_out = 0;
    const unsigned grid = (unsigned)ctx->num_cus * 8;
    const uint64_t n_part = (uint64_t)grid * kWaves;
    DevMem ctr, part, binfo, bslots;
    DT_TRY(dev_alloc(ctx, ctr, 256));
    DT_TRY(dev_alloc(ctx, part, n_part * 8 * sizeof(int64_t)));
    if (n) DT_TRY(build_bitmaps(g, binfo, bslots));
    FusedArgs fa{};
    fa.eoff = g->eoff.as<uint32_t>();
    fa.key = g->key.as<uint64_t>();
    fa.q = q;
    fa.u = cdev::unit_query(q);
    fa.unit_ok = g->span <= kUnitMaxSpan ? 1u : 0u;
    fa.cap_l = g->light_cap_used ? g->light_cap_used : 4;
    fa.shift = g->shift;
    fa.part = part.as<int64_t>();
    // the rest list: sized at an eighth of the static pairs, the pass runs again when it overflows
    uint64_t rcap = std::max<uint64_t>(g->m_s / 8, 1ull << 16);
    for (int attempt = 0; attempt < 2; ++attempt) {
        DT_TRY(dev_alloc(ctx, rest, rcap * 12));
        // counters: [0] next ticket (32-bit), [1] triangles, [2] candidates, [3] rest, [4..5] sum of products
        DT_HIP(hipMemsetAsync(ctr.ptr, 0, 64, st));
        unsigned long long *c64 = reinterpret_cast<unsigned long long *>(ctr.as<uint8_t>() + 8);
        fa.rest = rest.as<uint32_t>();
        fa.rest_cap = rcap;
        fa.rest_n = c64 + 2;
        fa.s3 = c64 + 3;
        prof_begin(ctx, kProfTriFill, st);
        if (n)
            k_tri<true><<<grid, kBlock, 0, st>>>(n, g->dag_row.as<uint32_t>(), g->dag_col.as<uint32_t>(), nullptr, 0,
                                                 c64, ctr.as<unsigned>(), c64 + 1, fa, binfo.as<uint4>(),
                                                 bslots.as<uint64_t>(), nullptr, 0);
        else
            DT_HIP(hipMemsetAsync(part.ptr, 0, n_part * 8 * sizeof(int64_t), st));
        prof_end(ctx, kProfTriFill, st);
        DT_HIP(hipGetLastError());
        uint64_t h[5] = {0, 0, 0, 0, 0};
        DT_HIP(hipMemcpyAsync(h, c64, 40, hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
        if (h[2] <= rcap) {
            *ntri_out = h[0];
            *cand_out = h[1];
            *n_rest = h[2];
            g->sum_sigma3 = ((unsigned __int128)h[4] << 64) | h[3];
            count_reduce(n_part, part.as<int64_t>(), out8_dev, st);
            return DT_OK;
        }
        rcap = h[2];
        rest.reset();
    }
    return fail(DT_EDEVICE, "triangle enumeration changed between passes");
}

}  // namespace dt
