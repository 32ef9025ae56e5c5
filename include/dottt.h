/*
 * dottt.h — C ABI of an MI355X (gfx950) library that counts (delta13, delta12, delta23)-temporal
 * triangles of a directed temporal multigraph exactly, per triangle type, after Pashanasangi &
 * Seshadhri, "Faster and Generalized Temporal Triangle Counting, via Degeneracy Ordering"
 * (KDD 2021).
 *
 * Conventions for every call:
 *   - The return value is DT_OK (0) or a negative DT_E* code; nothing is thrown across the ABI.
 *     dt_last_error() gives a human-readable message for the calling thread's last failure.
 *   - Pointers documented as "host" are ordinary host memory; "device" pointers are HIP device
 *     memory of the context's device (for example torch.cuda tensors' data_ptr()).
 *   - Inputs are copied; the library never keeps a caller pointer after a call returns.
 *   - Outputs go to caller-owned buffers.  Handles (dt_ctx, dt_graph, dt_server) own the device
 *     memory they allocate until the matching *_destroy / *_free / *_stop call.
 *   - Counts are exact int64.  out[k] is the count of type T(k+1) of Figure 2 (Section 1.1).
 *     A graph whose sum over static triangles of the product of the three pairs' multiplicities
 *     (sum_sigma3 in dt_stats, the count of every type together at infinite deltas) reaches
 *     2^63 is counted in 128 bits by dt_count, dt_count_visits and dt_count_oneshot, which
 *     return DT_EOVERFLOW (output untouched) only when a type's count reaches 2^63; the other
 *     count calls refuse such a graph with DT_EOVERFLOW before any work.
 *   - A dt_ctx and the graphs made from it are used by one host thread at a time; the dt_server_*
 *     calls are safe to call from any number of threads.
 *
 * Reading of the paper fixed by this library (the paper assumes distinct timestamps, Section 1.1
 * and Section 3, and says equal ones are allowed without defining them):
 *   - edges are ordered by the key (t, input index): equal timestamps follow input order;
 *     delta limits compare timestamps t;
 *   - self-loops (src == dst) are dropped at load; identical (u, v, t) edges are distinct edges;
 *   - a window [t_lo, t_hi] (inclusive) restricts all three edges of a triangle to it, which is
 *     the same as counting the graph filtered to the window.
 */
#ifndef DOTTT_H
#define DOTTT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DT_OK         0
#define DT_EINVAL   (-22)   /* bad argument: null pointer, node id >= n, negative delta, t_lo > t_hi */
#define DT_ENOMEM   (-12)   /* device allocation failed or would exceed the context's HBM budget   */
#define DT_EOVERFLOW (-75)  /* a size limit of this version, or a count that does not fit in int64  */
#define DT_EBUSY    (-16)   /* server full / graph busy                                             */
#define DT_ETIMEDOUT (-110) /* dt_server_wait timed out                                             */
#define DT_EDEVICE   (-5)   /* a HIP runtime error                                                  */
#define DT_ENOTBUILT (-38)  /* the graph has not been through dt_graph_build                        */

#define DT_INF INT64_MAX    /* a delta that behaves as infinity (any delta >= the graph's span does) */

typedef struct dt_ctx dt_ctx;
typedef struct dt_graph dt_graph;
typedef struct dt_server dt_server;

/* A count query (Definition 1, Section 1.1): a triple (e1, e2, e3) with e1 < e2 < e3 counts when
 * t2 - t1 <= d12, t3 - t2 <= d23 and t3 - t1 <= d13.  Deltas must be >= 0; the library rewrites
 * them to the equivalent triple d12' = min(d12, d13), d23' = min(d23, d13),
 * d13' = min(d13, d12' + d23'), which defines the same triangles and is what the per-ordering
 * counting procedures (Section 5, Appendix A) assume.  [t_lo, t_hi] is an inclusive window;
 * INT64_MIN..INT64_MAX is the whole graph. */
typedef struct {
    int64_t d13, d12, d23;
    int64_t t_lo, t_hi;
} dt_query;

/* Graph statistics; the first block mirrors the columns of Table 1 (Section 6). */
typedef struct {
    uint64_t n;                    /* vertices (ids 0..n-1)                                       */
    uint64_t m;                    /* temporal edges passed to dt_graph_load                      */
    uint64_t m_loaded;             /* temporal edges kept (self-loops dropped)                    */
    uint64_t self_loops_dropped;
    uint64_t m_static;             /* pairs joined by at least one temporal edge (Section 3)     */
    uint64_t n_static_triangles;   /* after dt_graph_build, else 0                                */
    uint32_t degeneracy;           /* after dt_graph_build: max core number (Definition, Sec. 3) */
    uint32_t max_multiplicity;     /* most temporal edges on one pair, both directions           */
    int64_t  t_min, t_max;         /* over kept edges                                             */
    /* build products (after dt_graph_build) */
    uint32_t max_out_degree;       /* of the orientation; at most the degeneracy                  */
    uint32_t peel_rounds;          /* removal rounds of the parallel core peel                    */
    uint64_t sum_sigma3_lo, sum_sigma3_hi; /* sum over static triangles of the product of the
                                              three pair multiplicities, 128-bit                  */
    uint64_t n_light_triangles, n_heavy_triangles; /* split chosen by the scheduler; a contested
                                                      triangle is in both medium and heavy lists */
    uint64_t n_medium_triangles;
    uint64_t n_unit_triangles;     /* one temporal edge on each pair, stored as 16-byte records   */
    uint64_t alg_bytes;            /* algorithmic bytes of one whole-graph count: 16 per unit
                                      triangle, else 12 + 36 + 8 (s_uv + s_uw)
                                      + 8 min(s_vw, 2 ceil(log2(s_vw+1)))                          */
    uint64_t alg_bytes_light;      /* the part of alg_bytes on light triangles                    */
    uint64_t alg_bytes_medium;     /* the part of alg_bytes on medium triangles                   */
    uint64_t alg_bytes_unit;       /* the part of alg_bytes on unit triangles                     */
    uint64_t alg_bytes_peel;       /* 16 n + 16 m_static: CSR and state read once, one update per pair */
    uint64_t alg_bytes_triangles;  /* 4 (m_static + candidates) + 12 per triangle written         */
    uint64_t tri_candidates;       /* (v, w) candidates tested: sum over v of d-(v) d+(v)          */
    uint64_t heavy_slots;          /* prefix-array slots of the heavy path                        */
    double   ms_load, ms_peel, ms_orient, ms_triangles, ms_schedule; /* phase wall times          */
    /* the count split and geometry the last build used */
    uint64_t n_contested_triangles; /* split between the medium path and the prefix procedures
                                       by each query's d13 (counted in n_medium and n_heavy)     */
    uint32_t light_pair_cap_used, medium_cost_pct_used;
    uint32_t light_blocks_per_cu, medium_blocks_per_cu;
    uint32_t autotuned;            /* 1: the values above came from the autotuner                 */
    uint32_t reserved0;
} dt_stats;

/* Tuning of the count scheduler.  A static triangle with one temporal edge on each pair (a unit
 * triangle) is stored with its ordering and orientation decided (Figures 3 and 4) and counted by
 * testing its three times against the query (when the graph's time span is below 2^31).  Any other
 * triangle whose two source-incident pairs carry P = sigma_uv * sigma_uw temporal-edge pairs is
 * counted by one lane enumerating those pairs (the pairwise form of Lemma 1) when
 * P <= light_pair_cap and the {v,w} pair carries at most 64 edges.  The rest are split between two
 * exact methods by a cost model with the query's d13 in it: the medium path (one lane per edge of
 * the smaller source-incident pair, walking only the edges of the other pair within d13 of it,
 * whose number grows with d13) and the prefix-count procedures of Algorithms 1-3 (Section 5, work
 * (sigma_uv + sigma_uw) log sigma whatever the deltas).  At build time each such triangle gets the
 * largest d13 (a power of two minus one) at which its close pairs stay within the prefix
 * procedures' cost times medium_cost_pct / 100; a query takes it on the medium path up to that d13
 * and on the prefix procedures beyond it, so no query does more than a constant times Theorem 1's
 * work on it.  Zero fields keep the default (light_pair_cap and medium_cost_pct: the autotuner's
 * choice for graphs of this size on this device, see dt_graph_build); force_path 1-3 sends every
 * triangle, unit ones included, down one path. */
typedef struct {
    uint32_t light_pair_cap;       /* 0 (default): the autotuner's choice, else 4                 */
    uint32_t heavy_chunk;          /* default 256 (the only compiled value)                       */
    uint32_t medium_pair_cap;      /* default 2^27, at most 2^30: larger P always takes the
                                      prefix procedures                                           */
    uint32_t force_path;           /* 0: split by the caps; 1: every triangle light;
                                      2: every triangle heavy; 3: every triangle medium
                                      (diagnostics and tests)                                     */
    uint32_t peel_tail;            /* the level peel hands the last peel_tail vertices to one
                                      workgroup (default and at most 16320; 1 keeps every level
                                      on the whole grid); read by the next dt_graph_build        */
    uint32_t order_method;         /* 0: the level-by-level core peel (default); 1: core numbers
                                      by h-index iteration, then every shell peeled at once.
                                      Both give the exact core numbers and an ordering with at
                                      most core(v) neighbours after each v; read by the next
                                      build or one-shot count                                    */
    uint32_t medium_cost_pct;      /* weight of the prefix procedures' cost against the medium
                                      path's, in percent (0: the autotuner's choice, else 100)    */
    uint32_t autotune;             /* 0: tune on the first build of a graph of this size class
                                      on this device (graphs of at least 2^20 static triangles;
                                      smaller ones take the defaults); 1: never tune; 2: tune
                                      again at the next build                                     */
} dt_tuning;

const char *dt_strerror(int code);
/* Message of the calling thread's last failed call ("" if none). */
const char *dt_last_error(void);

/* Context on HIP device `hip_device`.  hbm_budget_bytes caps the device memory the context's
 * graphs may hold (0 = no cap beyond the device).  Creates one HIP stream that all synchronous
 * calls use. */
int dt_ctx_create(int hip_device, uint64_t hbm_budget_bytes, dt_ctx **out);
int dt_ctx_destroy(dt_ctx *ctx);
/* Device memory currently held by the context's graphs and scratch. */
int dt_ctx_memory(const dt_ctx *ctx, uint64_t *used_bytes, uint64_t *budget_bytes);

/* Load a temporal graph (Section 3: a collection of m directed temporal edges (u, v, t)).
 * src, dst (uint32, < n) and t (int64) are host arrays of m entries; input position is the
 * tie-break of equal timestamps.  Extracts the static graph G (its pairs, Section 3) and groups
 * the temporal edges by pair and direction in key order (the CSR store of Section 4).
 * Limits of this version: m < 2^31, and (t_max - t_min) < 2^(64 - ceil(log2 m)) - 1 (so that a
 * timestamp and an input index pack into one 64-bit key); otherwise DT_EOVERFLOW. */
int dt_graph_load(dt_ctx *ctx, uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst,
                  const int64_t *t, dt_graph **out);
/* The same with src, dst and t already in device memory of the context's device. */
int dt_graph_load_device(dt_ctx *ctx, uint32_t n, uint64_t m, const uint32_t *src_dev,
                         const uint32_t *dst_dev, const int64_t *t_dev, dt_graph **out);

/* Degeneracy ordering by a parallel k-core peel (Section 3, Definitions of degeneracy and of the
 * degeneracy ordering), orientation of G into the DAG G_prec (Section 3), static triangle
 * enumeration in G_prec (Section 5, and the proof of Theorem 1), and the count schedule.  The
 * triangle list stays resident for every later count.  May be called again to rebuild. */
int dt_graph_build(dt_graph *g);
int dt_graph_set_tuning(dt_graph *g, const dt_tuning *tuning);
int dt_graph_stats(const dt_graph *g, dt_stats *out);

/* Per-type counts of (d13, d12, d23)-temporal triangles (Algorithm 4, Section 5): for every
 * static triangle <u, v, w> with u first in the ordering, every temporal ordering (Figure 3) and
 * orientation (Figure 4) is counted (Algorithms 1-3) and added to the type given by Table 2.
 * out: host int64[8].  Synchronous on the context's stream.  Counts in 128 bits when the graph's
 * sum_sigma3 reaches 2^63; DT_EOVERFLOW if a type's count reaches 2^63. */
int dt_count(dt_graph *g, const dt_query *q, int64_t out[8]);
/* The same, enqueued on `hip_stream` (a hipStream_t; NULL = the context's stream).  out8 is
 * device memory or pinned host memory that stays valid until the stream reaches the work.  A graph
 * whose sum_sigma3 reaches 2^63 is refused (DT_EOVERFLOW): the result is never read back, so there
 * is no point at which a type count beyond int64 could be reported. */
int dt_count_async(dt_graph *g, const dt_query *q, int64_t *out8, void *hip_stream);
/* dt_count_async without any allocation, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The same counts,
 * enqueued on `hip_stream` (NULL = the context's stream) into out8 (device or pinned host memory,
 * int64[8]), but the count's scratch -- per-block partial sums and the heavy path's prefix arrays --
 * lives in one fixed 64 MiB device array per GPU, held until the process ends, instead of memory
 * the context allocates.  A count that needs more scratch than that (a graph with many
 * prefix-count triangles) returns DT_ENOMEM and enqueues nothing.  Every call on one GPU shares
 * the array: calls whose work overlaps on the device (other streams, other threads, other
 * contexts on the same GPU) race and must be ordered by the caller. */
int dt_count_noalloc(dt_graph *g, const dt_query *q, int64_t *out8, void *hip_stream);
/* Diagnostic: dt_count with its kernels instrumented (slower).  *visits receives the work they
 * did in the units of Theorem 1's bound (Section 5): one per unit record tested, per (uv edge,
 * uw edge) pair evaluated on the light and medium paths, per outer edge of the medium path and per
 * source edge in each of the two passes of the prefix procedures.  With at most one cost-model
 * constant per triangle, visits stay within 2 * 48 * degeneracy * m', m' the temporal edges in the
 * window, for every d13.  out: host int64[8], equal to dt_count's (128-bit sums as dt_count). */
int dt_count_visits(dt_graph *g, const dt_query *q, int64_t out[8], uint64_t *visits);
/* Diagnostic: the 48 per-(ordering, orientation) counts, out[(pi-1)*8 + (rho-1)], with u, v, w
 * named by the degeneracy ordering (u first).  Sums of cells by Table 2 give dt_count's result. */
int dt_count_cells(dt_graph *g, const dt_query *q, int64_t out[48]);

/* One-shot count: the whole method for one query from the loaded graph -- degeneracy ordering,
 * orientation, and triangle enumeration that counts each triangle as it is found (Algorithm 4 with
 * the enumeration of Section 5 in one pass), without storing the triangle list: a triangle with
 * one temporal edge per pair is tested at once, a light one counted pairwise by its lane, and only
 * the few others are kept for the medium and heavy paths.  For graphs whose triangle list would
 * not fit and for single queries.  The result equals dt_count's.  Any earlier build is dropped
 * (dt_count then returns DT_ENOTBUILT until dt_graph_build); the graph's ordering is replaced.
 * out: host int64[8].  Synchronous on the context's stream.  The triangles kept for the medium
 * and heavy paths are counted in 128 bits when their sum_sigma3 reaches 2^63 (DT_EOVERFLOW if a
 * type's count reaches 2^63); the others are summed in int64, and a graph with so many triangles
 * that those sums could overflow (triangles * light_pair_cap * 64 >= 2^63) is refused. */
int dt_count_oneshot(dt_graph *g, const dt_query *q, int64_t out[8]);

/* A delta sweep on one graph (the parameter sweeps of Section 6, Figures 1 and 5): the counts of
 * k delta triples that share one window [t_lo, t_hi], out[8 j + i] = type i + 1 of queries[j],
 * equal to k separate dt_count calls.  Each pass over the triangles counts up to 8 triples, so
 * their records and lists are read from HBM once per 8 queries instead of once per query.
 * queries: host dt_query[k], k >= 1, all with the same t_lo and t_hi (otherwise DT_EINVAL);
 * out: host int64[8 k].  Synchronous on the context's stream. */
int dt_count_sweep(dt_graph *g, uint64_t k, const dt_query *queries, int64_t *out);

/* Batched counting: query i on graphs[i] for i < k (graphs may repeat), all in one persistent
 * launch over a shared work table.  out: host int64[k][8]. */
int dt_count_batch(dt_ctx *ctx, uint64_t k, dt_graph *const *graphs, const dt_query *queries,
                   int64_t (*out)[8]);

/* The item lengths of the context's last batched launch (out[0] light triangles per item, out[1]
 * medium entries per item), chosen by timing candidates on the first batch of each size class
 * (number of queries and their work, binary orders) on this device and cached for the process;
 * the server uses the same cache.  Host output uint32[2]. */
int dt_ctx_batch_tuning(const dt_ctx *ctx, uint32_t out[2]);

/* Diagnostics of the build products, for tests.  Host outputs.
 * dt_graph_order: core[v] (core number) and rank[v] (position of v in the ordering) for all n;
 * vertices removed in the same peel round may take their positions in a different order in
 * another build (any such order is a degeneracy ordering), and with them the names u, v, w of a
 * triangle's vertices that dt_count_cells uses.
 * dt_graph_triangles: the static triangles as node-id triples (a < b < c), in no fixed order;
 * writes min(count, cap) triples and sets *count (it runs the enumeration pass again). */
int dt_graph_order(const dt_graph *g, uint32_t *core, uint32_t *rank);
int dt_graph_triangles(const dt_graph *g, uint32_t *out, uint64_t cap, uint64_t *count);

int dt_graph_free(dt_graph *g);

/* Diagnostics: when profiling is on, the library records HIP events on the stream each kernel is
 * launched on, around the main kernels of the last build and the last count of the context:
 *   ms[0] core peel on the cooperative grid, ms[1] store re-layout, ms[2] triangle count pass,
 *   ms[3] triangle fill pass, ms[4] light count, ms[5] heavy prefix pass, ms[6] heavy count pass,
 *   ms[7] final reduction, ms[8] medium count, ms[9] unit-triangle count, ms[10] the peel's
 *   local adjacency of its last vertices, ms[11] the peel's one-workgroup finish, ms[12] core
 *   numbers and shell rounds (order_method 1; ms[0], ms[10] and ms[11] belong to method 0).
 * dt_ctx_last_profile waits for those events and reports their elapsed times (0 if not run). */
#define DT_PROFILE_SLOTS 13
int dt_ctx_set_profiling(dt_ctx *ctx, int enable);
int dt_ctx_last_profile(dt_ctx *ctx, float ms[DT_PROFILE_SLOTS]);

/* Serving: a request loop that keeps graphs resident in HBM and batches count queries of
 * differing deltas and windows into running device work (continuous batching). */
typedef struct {
    uint64_t hbm_budget_bytes;     /* memory the served graphs may hold (0 = the context's)        */
    uint32_t max_inflight_queries; /* queries admitted to the device at once (0 = 4096)            */
    uint32_t max_batch;            /* queries per device launch (0 = 512)                          */
    int64_t  deadline_ns;          /* per-query deadline; 0 = none                                 */
    uint32_t swap_to_host;         /* 1: graphs beyond the budget wait in host memory (below)      */
    uint32_t reserved;             /* 0                                                            */
} dt_server_cfg;

int dt_server_start(dt_ctx *ctx, const dt_server_cfg *cfg, dt_server **out);
/* Admit a built graph.  A graph's device bytes are its arrays plus the heavy path's scratch of one
 * query (dt_server_graph_info).  Without swap_to_host, DT_ENOMEM if it does not fit the budget
 * next to the graphs already admitted.  With swap_to_host, any graph that fits the budget alone
 * is admitted: if there is no room, its arrays are copied to host memory (pageable, owned by the
 * graph) and its HBM freed at once; when a query needs a graph that is in host memory, the server
 * moves the least recently used resident graphs that no batch on the device is using out to host
 * memory until it fits, then copies it back (byte for byte: its ordering and schedule are kept).
 * While such a server holds a graph, every other call that touches its device memory returns
 * DT_EBUSY (dt_graph_stats still answers); after dt_server_stop a graph left in host memory
 * returns to HBM on its next use.  The server does not take ownership: free the graph only after
 * dt_server_stop. */
int dt_server_add_graph(dt_server *s, dt_graph *g, uint32_t *graph_id);
int dt_server_submit(dt_server *s, uint32_t graph_id, const dt_query *q, uint64_t *ticket);
/* Wait for a ticket's counts; timeout_ns < 0 waits forever.  DT_ETIMEDOUT leaves the ticket
 * pending.  Each ticket can be waited for once. */
int dt_server_wait(dt_server *s, uint64_t ticket, int64_t out[8], int64_t timeout_ns);
/* Diagnostics of a server, host output: admitted graphs, those in HBM and their bytes (counted
 * against budget_bytes), graphs moved to host memory and back so far with their bytes, and the
 * queries answered (with any result code). */
typedef struct {
    uint64_t graphs, resident_graphs, resident_bytes, budget_bytes;
    uint64_t swap_outs, swap_ins, swap_out_bytes, swap_in_bytes;
    uint64_t queries_done;
} dt_server_info;
int dt_server_stats(dt_server *s, dt_server_info *out);
/* Whether graph_id's arrays are in HBM now (*resident 1) and its device bytes as admitted. */
int dt_server_graph_info(dt_server *s, uint32_t graph_id, int *resident, uint64_t *bytes);
int dt_server_stop(dt_server *s);

#ifdef __cplusplus
}
#endif

#endif /* DOTTT_H */
