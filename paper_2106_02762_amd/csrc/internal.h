// Internal declarations of the MI355X temporal-triangle library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "dottt.h"

namespace dt {

constexpr size_t kPinnedStage = 512 * 1024;

// ------------------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------------------
int fail(int code, const char *fmt, ...);   // records the thread's message, returns code
void clear_error();

#define DT_HIP(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::dt::fail(DT_EDEVICE, "%s failed: %s (%s:%d)", #expr,                 \
                              hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)

#define DT_TRY(expr)                  \
    do {                              \
        int rc_ = (expr);             \
        if (rc_ != DT_OK) return rc_; \
    } while (0)

// ------------------------------------------------------------------------------------------------
// context and device memory with a budget
// ------------------------------------------------------------------------------------------------
// A device allocation owned by a context; released by reset() or the destructor.
// Device memory owned by one object.  A pooled block goes back to its context's cache when
// released and may be handed to the next allocation at once: pooled memory must only be used in
// stream order on the context's own stream (build products and build temporaries).  Memory used
// on other streams (batch runners, scratch shared with foreign streams) is not pooled.
struct DevMem {
    dt_ctx *ctx = nullptr;
    void *ptr = nullptr;
    size_t bytes = 0;
    bool pooled = false;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    DevMem(DevMem &&o) noexcept { *this = std::move(o); }
    DevMem &operator=(DevMem &&o) noexcept;
    ~DevMem() { reset(); }
    void reset();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

}  // namespace dt

namespace dt {
// scratch of one count in flight: per-block partial sums and the heavy path's prefix arrays
struct Scratch {
    DevMem partials, heavy_vals, sweep_partials;
};
struct BatchRunner;
// item lengths of the batched launch: light triangles and medium entries per table item (unit
// records: four times the light length)
struct BatchTune {
    uint32_t light_chunk = 8192, medium_group = 1024;
};
}  // namespace dt

struct dt_ctx {
    int device = 0;
    uint64_t budget = 0;                 // 0 = no cap
    std::atomic<uint64_t> used{0};
    hipStream_t stream = nullptr;
    int num_cus = 0;
    // scratch reused by counts issued on the context's stream
    dt::Scratch scratch;
    dt::DevMem out8;
    dt::BatchRunner *batch = nullptr;        // dt_count_batch's runner (created on first use)
    dt::BatchTune batch_tune;                // item lengths of the last batch (autotuned per size class)
    int64_t *pinned_out = nullptr;       // 64 int64 of pinned host memory for results
    uint8_t *pinned_stage = nullptr;     // kPinnedStage bytes of pinned host memory for a build's read-backs
    hipEvent_t ev_a = nullptr, ev_b = nullptr;   // order foreign streams around the scratch
    // a count's light and medium kernels run on these, forked from and joined to the count's stream
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
    // a build's re-layout of the temporal store runs on side[0] next to the enumeration: fork, done
    hipEvent_t ev_relay[2] = {nullptr, nullptr};
    // optional per-kernel timing (dt_ctx_set_profiling)
    bool prof = false;
    hipEvent_t prof_ev[2 * DT_PROFILE_SLOTS] = {};
    bool prof_used[DT_PROFILE_SLOTS] = {};
    // cache of released pooled blocks (size -> address); counted in `used`
    std::mutex pool_mu;
    std::multimap<size_t, void *> pool;
    uint64_t pool_bytes = 0;
};

namespace dt {

// DT_ENOMEM on budget or HIP failure; see DevMem for when `pooled` is allowed
int dev_alloc(dt_ctx *ctx, DevMem &m, size_t bytes, bool pooled = true);
void pool_trim(dt_ctx *ctx, uint64_t keep_bytes);   // free cached blocks down to keep_bytes

// profiling marks around one kernel launch (no-ops unless profiling is on)
enum ProfSlot { kProfPeel = 0, kProfRelayout, kProfTriCount, kProfTriFill, kProfLight,
                kProfHeavyPrefix, kProfHeavyCount, kProfReduce, kProfMedium, kProfUnit, kProfPeelAdj,
                kProfPeelTail, kProfCore };
inline void prof_begin(dt_ctx *c, int slot, hipStream_t s) {
    if (c->prof) { (void)hipEventRecord(c->prof_ev[2 * slot], s); c->prof_used[slot] = true; }
}
inline void prof_end(dt_ctx *c, int slot, hipStream_t s) {
    if (c->prof) (void)hipEventRecord(c->prof_ev[2 * slot + 1], s);
}
// a new build or count: its slots report 0 until its kernels record them
inline void prof_clear(dt_ctx *c, bool build) {
    static constexpr int kBuild[] = {kProfPeel, kProfRelayout, kProfTriCount, kProfTriFill, kProfPeelAdj,
                                     kProfPeelTail, kProfCore};
    static constexpr int kCount[] = {kProfLight, kProfHeavyPrefix, kProfHeavyCount, kProfReduce, kProfMedium,
                                     kProfUnit};
    if (build)
        for (int s : kBuild) c->prof_used[s] = false;
    else
        for (int s : kCount) c->prof_used[s] = false;
}
int ensure(dt_ctx *ctx, DevMem &m, size_t bytes);   // grow-only, not pooled

// ------------------------------------------------------------------------------------------------
// query as the kernels see it: deltas rewritten and clamped, window in key space
// ------------------------------------------------------------------------------------------------
struct DQuery {
    int64_t d13, d12, d23;   // 0 <= d12, d23 <= d13 <= d12 + d23 <= 2 * span
    uint64_t klo, khi;       // window as keys: kept iff klo <= key < khi
    int64_t span;            // t_max - t_min (relative times lie in [0, span])
    int shift;               // key = (t - t_min) << shift | input index
    int windowed;            // 0: klo = 0, khi = ~0
    uint32_t qlev;           // level of d13 (query_level): contested triangles of a lower level take
                             // the prefix procedures, the others the pairwise medium path
};

// Levels of the medium / heavy split.  A contested triangle's level l (1..31) says that its close
// pairs within D(l) = 2^(l-1) - 1 of each other fit its pair budget (the medium path's cost stays
// below the prefix procedures'); level 0: never, kLevelAlways: every query.  A query takes a
// contested triangle on the medium path iff its level is at least query_level(d13), the smallest
// l with D(l) >= d13 (32 when none).
constexpr uint32_t kLevels = 32;
constexpr uint8_t kLevelAlways = 255;
__host__ __device__ inline int64_t level_delta(uint32_t l) { return l == 0 ? -1 : (int64_t(1) << (l - 1)) - 1; }
__host__ __device__ inline uint32_t query_level(int64_t d13) {
    uint32_t l = 1;
    while (l < kLevels && level_delta(l) < d13) ++l;
    return l;
}

// Unit triangles: static triangles with exactly one temporal edge on each of their three pairs
// (the common case in sparse interaction data).  Their ordering pi (Figure 3) and orientation rho
// (Figure 4) do not depend on the query, so each is stored as one 16-byte record
//   x = t1, y = t2 - t1, z = t3 - t2, w = (cell << 8) | (type - 1)
// with times relative to t_min and cell = 8 (pi - 1) + (rho - 1); a query only tests its deltas
// and window against (x, y, z).  Used when the time span is below 2^31.  Records are grouped by
// t1 bucket (t1 >> unit_shift, at most 2^16 buckets) so that a window selects a contiguous range;
// the host keeps the bucket starts.
constexpr int64_t kUnitMaxSpan = (int64_t(1) << 31) - 1;
// Window index of the light and medium lists.  A triangle can hold a temporal triangle inside a
// window [lo, hi] only if each of its three pairs has an edge inside it, that is only if
// F <= hi and L >= lo, where F is the latest of the three pairs' first edge times and L the
// earliest of their last edge times.  Both are cut into kSlices time slices (relative time
// >> cell_shift, the last slice open-ended) and the lists are ordered by cell
// slice(F) * kSlices + slice(L), so a window selects at most kSlices contiguous ranges: for every
// slice f <= slice(hi), the cells (f, l) with l >= slice(lo).
constexpr int kSliceBits = 5;
constexpr uint32_t kSlices = 1u << kSliceBits;
constexpr uint32_t kCells = kSlices * kSlices;
// up to kSlices ranges [b[r], b[r] + pre[r + 1] - pre[r]) of a list; pre[0] = 0, pre[n] = total
struct Ranges {
    uint32_t n;
    uint64_t b[kSlices];
    uint64_t pre[kSlices + 1];
};

// ------------------------------------------------------------------------------------------------
// build products of one graph (all device arrays unless noted)
// ------------------------------------------------------------------------------------------------
// The medium list holds the always-medium triangles first, then the contested ones by descending
// level; the heavy list the contested ones in that same order, then the always-heavy ones.  So a
// whole-span query at level l walks a prefix of the medium list and a suffix of the heavy list,
// whose bounds the host keeps per level.
struct Schedule {
    uint64_t n_light = 0, n_medium = 0, n_heavy = 0, n_unit = 0;
    uint64_t n_always_medium = 0, n_contested = 0, n_always_heavy = 0;
    DevMem unit;                        // uint4[n_unit] unit-triangle records
    int unit_shift = 0;                 // t1 bucket of a record: t1 >> unit_shift
    std::vector<uint32_t> unit_index;   // host: first record of each t1 bucket, then n_unit
    DevMem light;       // uint32[3 * n_light]: (e_uv, e_uw, e_vw) DAG edge ids
    DevMem medium;      // uint32[3 * n_medium]
    DevMem mitems;      // uint32[2 * n_mitems]: (medium triangle, outer edge and inner chunk) entries
    uint64_t n_mitems = 0;
    // windowed copies of light, medium and mitems in window-cell order (the originals keep the
    // enumeration order, whose locality the whole-span count needs)
    DevMem light_w, medium_w, mitems_w;
    int cell_shift = 0;                 // time slice of the window index: t >> cell_shift
    std::vector<uint64_t> light_cells;  // host: first entry of light_w in each cell, then n_light
    std::vector<uint64_t> mitem_cells;  // host: first entry of mitems_w in each cell, then n_mitems
    DevMem heavy;       // uint32[3 * n_heavy]
    DevMem hslot;       // uint64[n_heavy + 1]: first scratch slot of each heavy triangle
    uint64_t n_slots = 0;
    DevMem chunks;      // uint32[2 * n_chunks]: (heavy triangle, first element) per work item
    uint64_t n_chunks = 0;
    DevMem pchunks;     // uint32[2 * n_pchunks]: (heavy triangle, first | list) per prefix chunk
    uint64_t n_pchunks = 0;
    DevMem mlev_w;      // uint8[n_medium]: level of each triangle of medium_w
    // per query level l = 1..kLevels (entry 0 unused): first medium entry not walked by a whole-span
    // query; first heavy triangle, count chunk, prefix chunk and prefix slot it counts
    uint64_t med_item_at[kLevels + 1] = {}, heavy_tri_at[kLevels + 1] = {}, heavy_chunk_at[kLevels + 1] = {},
             heavy_pchunk_at[kLevels + 1] = {}, heavy_slot_at[kLevels + 1] = {};
};

// Per-graph count geometry (blocks per compute unit of the light and medium kernels), chosen by the
// autotuner or the defaults.
struct CountGeom {
    uint32_t light_bpc = 16, medium_bpc = 8;
};

}  // namespace dt

struct dt_graph {
    dt_ctx *ctx = nullptr;
    uint32_t n = 0;
    uint64_t m_in = 0, m = 0, self_loops = 0, m_s = 0;
    int64_t t_min = 0, t_max = 0, span = 0;
    int shift = 0;
    uint32_t max_mult = 0;
    // load products
    dt::DevMem sx, sy;          // uint32[m_s]: pair endpoints x < y
    dt::DevMem row;             // uint32[n + 1]: undirected CSR of G
    dt::DevMem col, ceid;       // uint32[2 m_s]: neighbour, pair id
    dt::DevMem psid;            // uint32[m]: pair of each temporal edge (pair-major, key order)
    dt::DevMem pdir;            // uint8[m]: 0 if the edge goes x -> y
    dt::DevMem pkey;            // uint64[m]: key of each temporal edge (same order)
    dt::DevMem pstart;          // uint32[m_s + 1]: first edge of each pair in that order
    dt::DevMem c1;              // uint32[m + 1]: edges with pdir = 1 before each position
    // build products
    bool built = false;
    uint32_t kappa = 0, max_outdeg = 0, peel_rounds = 0;
    dt::DevMem core, rank, order;  // uint32[n]: core number, position in the ordering, vertex at position
    dt::DevMem dag_row;         // uint32[n + 1]: out-CSR of G_prec in rank space
    dt::DevMem dag_col;         // uint32[m_s]: head rank of each DAG edge
    dt::DevMem eoff;            // uint32[2 m_s + 1]: DAG edge d: tail->head edges [eoff[2d], eoff[2d+1]),
                                //                    head->tail edges [eoff[2d+1], eoff[2d+2])
    dt::DevMem key;             // uint64[m]: keys in that layout
    bool relay_pending = false; // key is still being written on the context's side[0] stream
    dt::DevMem relay_tmp[4];    // inputs and temporaries of that re-layout, held until it is joined
    uint64_t n_tri = 0;
    uint64_t n_tri_list = 0;    // entries of the triangle list the last schedule was made from (with empty ones)
    unsigned __int128 sum_sigma3 = 0;
    uint64_t alg_bytes = 0, alg_bytes_light = 0, alg_bytes_medium = 0, alg_bytes_peel = 0, alg_bytes_tri = 0;
    uint64_t alg_bytes_unit = 0;
    uint64_t tri_candidates = 0;
    dt::Schedule sched;
    dt::CountGeom geom;
    // the user's tuning (zero fields: automatic) and the values the last build used
    dt_tuning tuning{0, 256, 1u << 27, 0, 0, 0, 0, 0};
    uint32_t light_cap_used = 0, cost_pct_used = 0;
    int tuned = 0;              // 1: the build's split and geometry came from the autotuner
    double ms_load = 0, ms_peel = 0, ms_orient = 0, ms_tri = 0, ms_sched = 0;
    // host copies of the device arrays (in graph_arrays order) while the graph is out of HBM
    std::vector<std::unique_ptr<uint8_t[]>> swap_host;
    std::vector<size_t> swap_bytes;
    bool swapped = false;
    dt_server *held_by = nullptr;   // a server that swaps graphs holds its graphs until it stops
};

namespace dt {

// the autotuner's choices for one size class of graphs on one device (tune.hip)
struct TunedCount {
    uint32_t light_cap = 4, cost_pct = 100, light_bpc = 16, medium_bpc = 8;
};
bool tuned_lookup(const dt_graph *g, TunedCount *t);
// times candidate splits and geometries of g's count (building a schedule from tri for each),
// caches the best for g's size class and leaves g's split and geometry set to it (the schedule
// must be built again)
int autotune_count(dt_graph *g, DevMem &tri, TunedCount *out);

// build phases (each returns a DT_* code)
int load_graph(dt_graph *g, const uint32_t *src_dev, const uint32_t *dst_dev, const int64_t *t_dev);
int peel(dt_graph *g);         // level-by-level core peel (order_method 0)
int core_order(dt_graph *g);   // h-index core numbers, then shell rounds (order_method 1)
int order_vertices(dt_graph *g);   // the ordering by the graph's order_method
int orient(dt_graph *g, bool overlap = false);   // overlap: re-layout on side[0], see relayout_join
// an empty entry of a triangle list (all three DAG edge ids): the enumeration leaves some, the
// schedule skips them
constexpr uint32_t kNoEdge = 0xffffffffu;
// every static triangle as (e_uv, e_uw, e_vw) DAG edge ids, in a list of *nlist entries of which
// *ntri are triangles and the others empty; *cand: candidates tested
int enumerate_triangles(const dt_graph *g, DevMem &tri, uint64_t *ntri, uint64_t *cand, uint64_t *nlist);
// the schedule of g's count from its triangle list tri (g->n_tri_list entries, g->n_tri triangles)
int make_schedule(dt_graph *g, DevMem &tri);
// orders the context's stream after a re-layout that orient(g, true) left running on side[0]
// (no-op otherwise) and releases its temporaries; to be called before anything reads g->key
int relayout_join(dt_graph *g);
// One-shot pass: enumerate the triangles of the oriented graph and count the unit and light ones
// for query q as they are found (sum to out8_dev); the others go to `rest` (*n_rest triangles,
// three DAG edge ids each).  *ntri: all static triangles; *cand: candidates tested; g->sum_sigma3:
// the sum of multiplicity products over all of them.
int fused_count(dt_graph *g, const DQuery &q, int64_t *out8_dev, DevMem &rest, uint64_t *n_rest, uint64_t *ntri,
                uint64_t *cand);
// unit records [*b, *e) that can hold triangles inside the query's window (all when unwindowed)
void unit_range(const dt_graph *g, const DQuery &q, uint64_t *b, uint64_t *e);
// the ranges of a cell-ordered list (cell starts ix, kCells + 1 entries) that can hold triangles
// inside the query's window (the whole list when unwindowed)
void cell_ranges(const std::vector<uint64_t> &ix, int cell_shift, const DQuery &q, Ranges &r);

// counting
int normalise_query(const dt_graph *g, const dt_query *q, DQuery *out, bool *empty);
// Device scratch of one count: per-block partial sums and the heavy path's prefix arrays.
struct ScratchView {
    int64_t *part = nullptr;
    size_t part_bytes = 0;
    uint8_t *heavy = nullptr;
    size_t heavy_bytes = 0;
};
// The heavy triangles a query counts: [hb, hb + n) of the heavy list, their count chunks from cb,
// prefix chunks from pb and prefix slots from slot_base; scratch_bytes of prefix arrays, chunk
// totals and clipped bounds.
struct HeavyRange {
    uint64_t hb = 0, n = 0, cb = 0, pb = 0, slot_base = 0;
    size_t scratch_bytes = 0;
};
void heavy_range(const dt_graph *g, const DQuery &q, HeavyRange &h);
namespace cdev { struct HeavyArgs; }
using cdev::HeavyArgs;
// the arguments of a query's heavy kernels over the range hr, with its scratch at `scratch`
void heavy_args(const dt_graph *g, const DQuery &q, const HeavyRange &hr, uint8_t *scratch, HeavyArgs &A);
// The medium entries a query walks (whole span: a prefix by its level; windowed: the window cells,
// with *lev the per-triangle levels to check).
void medium_ranges(const dt_graph *g, const DQuery &q, Ranges &r, const uint8_t **lev);
// Launch geometry of one count and the scratch it needs (count_plan, host only).
struct CountPlan {
    Ranges lr, mr;                               // light triangles and medium entries the query sees
    const uint8_t *mlev = nullptr;               // levels of the windowed medium copy (or null)
    HeavyRange hr;
    const uint32_t *light = nullptr, *medium = nullptr, *mitems = nullptr;
    unsigned lg = 0, hg = 0, mg = 0, ug = 0;     // grids of the light, heavy, medium and unit kernels
    uint64_t ub = 0, ue = 0;                     // unit records [ub, ue)
    uint64_t n_part = 0;                         // partial slots
    size_t part_bytes = 0, heavy_bytes = 0;
    unsigned parts = 15;
    bool wide = false;   // 128-bit counts: the result is 16 words, (low, high) per type
};
void count_plan(const dt_graph *g, const DQuery &q, unsigned parts, CountPlan &p);
// Enqueue a planned count on stream s with scratch sv (which must hold the plan's needs).
int count_launch(dt_graph *g, const DQuery &q, const CountPlan &p, int64_t *out8_dev, hipStream_t s, bool cells,
                 int64_t *cells_dev, const ScratchView &sv, unsigned long long *visits = nullptr);
// Enqueue one count on stream s using scratch sc (grown as needed).  parts: bit 0 light, bit 1 medium, bit 2 heavy,
// bit 3 unit (all = 15).  Without cells the sum of the selected parts goes to out8_dev (int64[8]); with cells
// the 48 cells are accumulated into cells_dev (zeroed here).
int count_enqueue(dt_graph *g, const DQuery &q, int64_t *out8_dev, hipStream_t s, bool cells,
                  int64_t *cells_dev, Scratch &sc, unsigned parts = 15, unsigned long long *visits = nullptr);
// The no-allocation count's scratch: noalloc_init takes the current device's address of it (once
// per device, from the context's setup); noalloc_capacity is its size in bytes.
int noalloc_init(int device);
size_t noalloc_capacity();
// sum of n_part int64[8] partials into out8_dev, on stream s
void count_reduce(uint64_t n_part, const int64_t *part, int64_t *out8_dev, hipStream_t s);
// delta triples counted in one pass of a sweep
constexpr uint32_t kSweepMax = 8;
// Enqueue the counts of k <= kSweepMax queries that share one window (and so one set of list
// ranges) in one pass over the triangles: out_dev[8 j + i] = type i + 1 of query j.
int count_sweep_enqueue(dt_graph *g, const DQuery *qs, uint32_t k, int64_t *out_dev, hipStream_t s, Scratch &sc);
void destroy_batch_runner(BatchRunner *r);
int make_batch_runner(dt_ctx *ctx, BatchRunner **out);
// plan the item table of k queries and enqueue it on the runner's stream (asynchronous)
int batch_plan_and_launch(BatchRunner *r, uint64_t k, dt_graph *const *graphs, const DQuery *qs,
                          const bool *empty, const BatchTune &bt);
// the item lengths for this batch's size class on this device: cached, or timed on this batch with
// runner r (whose stream must be idle) and cached
int batch_tuned(dt_ctx *ctx, BatchRunner *r, uint64_t k, dt_graph *const *graphs, const DQuery *qs,
                const bool *empty, BatchTune *out);
int batch_wait(BatchRunner *r, uint64_t k, const bool *empty, int64_t (*out)[8]);
bool batch_ready(BatchRunner *r);
int batch_sync(BatchRunner *r);
// the most vertices the level peel hands to its one-workgroup finish (the LDS of one workgroup
// holds their local CSR rows, degrees, queue and live list)
constexpr uint32_t kPeelTailMax = 16320;

struct DeviceGuard {   // make the context's device current for the duration of a call
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

uint64_t graph_device_bytes(const dt_graph *g);
// Moves every device array of g to host memory (copies on stream st, then frees the device
// memory) or back into HBM; g must have no device work outstanding.  On failure g is left as it
// was.  graph_swap_in of a resident graph does nothing.
int graph_swap_out(dt_graph *g, hipStream_t st);
int graph_swap_in(dt_graph *g, hipStream_t st);
// The checks every call on a graph makes: not null; built if need_built; and, when the call
// touches device memory (device), not held by a swapping server, and in HBM (a graph left in host
// memory by a stopped server is brought back here).
int check_graph(const dt_graph *g, bool need_built, bool device = true);
int count_batch(dt_ctx *ctx, uint64_t k, dt_graph *const *graphs, const dt_query *queries,
                int64_t (*out)[8]);

// library primitives (rocPRIM), out of place, enqueued on stream s; temporary storage is taken
// from the context's budget and released before returning.  Sorts always start at bit 0: on this
// rocPRIM a nonzero begin_bit gave unsorted output for mid-size inputs (its merge-sort path).
int sort_pairs_u64_u32(dt_ctx *ctx, const uint64_t *kin, uint64_t *kout, const uint32_t *vin,
                       uint32_t *vout, size_t n, int end_bit, hipStream_t s);
int sort_pairs_u64_u64(dt_ctx *ctx, const uint64_t *kin, uint64_t *kout, const uint64_t *vin,
                       uint64_t *vout, size_t n, int end_bit, hipStream_t s);
// (16-bit key, 16-byte record) pairs; with `keep` the temporary storage is handed to the caller
// instead of being released (and a foreign stream s is not waited for): for a sort left running on
// a side stream, whose caller releases it after the join
int sort_pairs_u16_u4(dt_ctx *ctx, const uint16_t *kin, uint16_t *kout, const uint4 *vin, uint4 *vout,
                      size_t n, int end_bit, hipStream_t s, DevMem *keep = nullptr);
// (keep: with a stream other than the context's, hand the temporary to the caller, who releases it
// after joining that stream, instead of waiting for the stream here)
int exclusive_scan_u32(dt_ctx *ctx, const uint32_t *in, uint32_t *out, size_t n, hipStream_t s,
                       DevMem *keep = nullptr);
int exclusive_scan_u64(dt_ctx *ctx, const uint64_t *in, uint64_t *out, size_t n, hipStream_t s);

// timing helper
double now_ms();

inline unsigned grid_for(uint64_t n, unsigned block) {
    uint64_t g = (n + block - 1) / block;
    if (g == 0) g = 1;
    if (g > 0x7fffffffull) g = 0x7fffffffull;
    return (unsigned)g;
}

}  // namespace dt
