/*
 * Plain CPU oracle for exact (delta13, delta12, delta23)-temporal triangle counts.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's CPU-baseline
 * leg may load, call or link this code.  It shares no code, header, table or helper with the GPU
 * library; the two never import each other.
 *
 * What it computes.  Definition 1 (Section 1.1) with the eight types of Figure 2:
 *   - keep the edges with src != dst and t_lo <= t <= t_hi;
 *   - give every kept edge the key (t, input index): equal timestamps are ordered by input position;
 *   - count every ordered triple e1 < e2 < e3 (by key) whose edges lie on the three distinct vertex
 *     pairs of one static triangle and satisfy t2 - t1 <= d12, t3 - t2 <= d23, t3 - t1 <= d13;
 *   - add each triple to its type (classify(), read off the eight panels of Figure 2) and to its
 *     cell (temporal order pi of Figure 3, orientation rho of Figure 4) relative to the triangle's
 *     vertices u < v < w taken in node-id order.
 * With distinct timestamps the key order is the timestamp order, so this is exactly Definition 1.
 * Types and cells are decoded separately, so that the paper's Table 2 (which maps a cell to a type)
 * can be checked against them rather than assumed.
 *
 * How.  No part of the paper's fast algorithm (Algorithms 1-4) is used.  Static triangles are listed
 * by the textbook rule "for each vertex x, test every two neighbours that come after x in
 * (degree, id) order for adjacency", which finds each triangle once.  For each triangle the kept
 * edges of its three pairs are merged by key; every e1 and every later e2 on another pair with
 * t2 - t1 <= d12 is paired, and the e3 on the remaining pair (one direction at a time) with
 * key > key(e2) and t3 <= min(t2 + d23, t1 + d13) are counted by two binary searches in that pair's
 * key-sorted edge list.  Work is O(sum over triangles of (pairs e1,e2 within d12) * log).
 *
 * Graph statistics (the columns of Table 1) come from the same edge grouping; the degeneracy and
 * core numbers use the bucket form of smallest-last vertex removal (Matula & Beck; Section 3).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-22)
#define OR_ENOMEM (-12)
#define OR_EOVERFLOW (-75)

typedef struct {
    uint64_t n, m, self_loops, m_window, m_static, n_triangles;
    uint32_t degeneracy, max_multiplicity;
    int64_t t_min, t_max;
    uint64_t sum_sigma3_lo, sum_sigma3_hi; /* sum over static triangles of the product of the three
                                              pair multiplicities (both directions), 128-bit */
} oracle_stats;

/* One kept temporal edge, stored with its unordered pair (a < b) and direction. */
typedef struct {
    uint32_t a, b;   /* a < b */
    int64_t t;
    uint32_t idx;    /* input position: the tie-break of equal timestamps */
    uint32_t dir;    /* 0: a -> b, 1: b -> a */
} edge_t;

typedef struct {
    uint32_t n;
    uint64_t m_in, self_loops, m;   /* m = kept edges */
    edge_t *e;                      /* sorted by (a, b, dir, t, idx) */
    uint64_t P;                     /* number of static pairs */
    uint32_t *pa, *pb;              /* pair endpoints */
    uint64_t *pbeg;                 /* pair p: dir 0 edges [pbeg[2p], pbeg[2p+1]), dir 1 [pbeg[2p+1], pbeg[2p+2]) */
    uint64_t *adj_off;              /* n+1 */
    uint32_t *adj_nbr, *adj_pair;   /* neighbours sorted by id */
    int64_t t_min, t_max;
} graph_t;

static int cmp_edge(const void *x, const void *y)
{
    const edge_t *p = (const edge_t *)x, *q = (const edge_t *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->dir != q->dir) return p->dir < q->dir ? -1 : 1;
    if (p->t != q->t) return p->t < q->t ? -1 : 1;
    if (p->idx != q->idx) return p->idx < q->idx ? -1 : 1;
    return 0;
}

static void graph_free(graph_t *g)
{
    free(g->e); free(g->pa); free(g->pb); free(g->pbeg);
    free(g->adj_off); free(g->adj_nbr); free(g->adj_pair);
    memset(g, 0, sizeof(*g));
}

static int graph_build(graph_t *g, uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst,
                       const int64_t *t, int64_t t_lo, int64_t t_hi)
{
    memset(g, 0, sizeof(*g));
    g->n = n;
    g->m_in = m;
    if (m && (!src || !dst || !t)) return OR_EINVAL;
    if (m >= ((uint64_t)1 << 32)) return OR_EINVAL;
    for (uint64_t i = 0; i < m; i++)
        if (src[i] >= n || dst[i] >= n) return OR_EINVAL;
    g->e = (edge_t *)malloc(sizeof(edge_t) * (m ? m : 1));
    if (!g->e) return OR_ENOMEM;
    uint64_t k = 0;
    g->t_min = INT64_MAX;
    g->t_max = INT64_MIN;
    for (uint64_t i = 0; i < m; i++) {
        if (src[i] == dst[i]) { g->self_loops++; continue; }
        if (t[i] < t_lo || t[i] > t_hi) continue;
        edge_t *x = &g->e[k++];
        x->a = src[i] < dst[i] ? src[i] : dst[i];
        x->b = src[i] < dst[i] ? dst[i] : src[i];
        x->dir = src[i] < dst[i] ? 0u : 1u;
        x->t = t[i];
        x->idx = (uint32_t)i;
        if (t[i] < g->t_min) g->t_min = t[i];
        if (t[i] > g->t_max) g->t_max = t[i];
    }
    g->m = k;
    qsort(g->e, k, sizeof(edge_t), cmp_edge);

    /* static pairs */
    uint64_t P = 0;
    for (uint64_t i = 0; i < k; i++)
        if (i == 0 || g->e[i].a != g->e[i - 1].a || g->e[i].b != g->e[i - 1].b) P++;
    g->P = P;
    g->pa = (uint32_t *)malloc(sizeof(uint32_t) * (P ? P : 1));
    g->pb = (uint32_t *)malloc(sizeof(uint32_t) * (P ? P : 1));
    g->pbeg = (uint64_t *)malloc(sizeof(uint64_t) * (2 * P + 1));
    g->adj_off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    g->adj_nbr = (uint32_t *)malloc(sizeof(uint32_t) * (P ? 2 * P : 1));
    g->adj_pair = (uint32_t *)malloc(sizeof(uint32_t) * (P ? 2 * P : 1));
    if (!g->pa || !g->pb || !g->pbeg || !g->adj_off || !g->adj_nbr || !g->adj_pair) return OR_ENOMEM;
    /* pair q: direction-0 edges [pbeg[2q], pbeg[2q+1]), direction-1 edges [pbeg[2q+1], pbeg[2q+2]) */
    uint64_t p = 0, i = 0;
    while (i < k) {
        uint64_t j = i;
        while (j < k && g->e[j].a == g->e[i].a && g->e[j].b == g->e[i].b) j++;
        uint64_t mid = i;
        while (mid < j && g->e[mid].dir == 0) mid++;
        g->pa[p] = g->e[i].a;
        g->pb[p] = g->e[i].b;
        g->pbeg[2 * p] = i;
        g->pbeg[2 * p + 1] = mid;
        p++;
        i = j;
    }
    g->pbeg[2 * P] = k;

    /* adjacency sorted by neighbour id: the entries where x is the larger endpoint (neighbours < x,
       appearing in increasing order because pairs are sorted by a) come first, then those where x
       is the smaller endpoint (neighbours > x, increasing). */
    for (uint64_t q = 0; q < P; q++) { g->adj_off[g->pa[q] + 1]++; g->adj_off[g->pb[q] + 1]++; }
    for (uint32_t v = 0; v < n; v++) g->adj_off[v + 1] += g->adj_off[v];
    uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)n + 1));
    if (!fill) return OR_ENOMEM;
    memcpy(fill, g->adj_off, sizeof(uint64_t) * ((size_t)n + 1));
    for (uint64_t q = 0; q < P; q++) {
        uint32_t x = g->pb[q];
        g->adj_nbr[fill[x]] = g->pa[q];
        g->adj_pair[fill[x]++] = (uint32_t)q;
    }
    for (uint64_t q = 0; q < P; q++) {
        uint32_t x = g->pa[q];
        g->adj_nbr[fill[x]] = g->pb[q];
        g->adj_pair[fill[x]++] = (uint32_t)q;
    }
    free(fill);
    return OR_OK;
}

/* pair id of {x, y}, or -1 */
static int64_t find_pair(const graph_t *g, uint32_t x, uint32_t y)
{
    uint64_t lo = g->adj_off[x], hi = g->adj_off[x + 1];
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (g->adj_nbr[mid] < y) lo = mid + 1; else hi = mid;
    }
    if (lo < g->adj_off[x + 1] && g->adj_nbr[lo] == y) return (int64_t)g->adj_pair[lo];
    return -1;
}

/* "x comes before y" in (degree, id) order */
static int before(const graph_t *g, uint32_t x, uint32_t y)
{
    uint64_t dx = g->adj_off[x + 1] - g->adj_off[x], dy = g->adj_off[y + 1] - g->adj_off[y];
    return dx < dy || (dx == dy && x < y);
}

/* Figure 2.  e1 = a -> b, c the third vertex; e2 = s2 -> d2, e3 = s3 -> d3. */
static int classify(uint32_t a, uint32_t b, uint32_t s2, uint32_t d2, uint32_t s3, uint32_t d3)
{
    if (s2 == b || d2 == b) {                 /* e2 on {b,c}, so e3 on {a,c} */
        int e3_from_a = (s3 == a);
        if (d2 == b) return e3_from_a ? 1 : 2; /* e2 = c -> b */
        return e3_from_a ? 3 : 4;              /* e2 = b -> c; T4 is the cycle a->b->c->a */
    }
    /* e2 on {a,c}, so e3 on {b,c} */
    int e3_into_b = (d3 == b);
    (void)s3;
    if (s2 == a) return e3_into_b ? 5 : 7;     /* e2 = a -> c */
    return e3_into_b ? 6 : 8;                  /* e2 = c -> a; T8 is the cycle a->b->c->a */
}

/* Figure 4: orientation index 1..8 from the directions of the uv, uw, vw edges
   (1 when the edge points from the smaller-named vertex of u < v < w). */
static int rho_index(int fwd_uv, int fwd_uw, int fwd_vw)
{
    static const int tab[2][2][2] = {
        /* fwd_uv = 0 */ { /* fwd_uw = 0 */ {6, 8}, /* fwd_uw = 1 */ {7, 5} },
        /* fwd_uv = 1 */ { /* fwd_uw = 0 */ {2, 4}, /* fwd_uw = 1 */ {3, 1} },
    };
    return tab[fwd_uv][fwd_uw][fwd_vw];
}

/* Figure 3: temporal order index 1..6 from the pair (0 = uv, 1 = uw, 2 = vw) holding e1 and e2. */
static int pi_index(int first, int second)
{
    if (first == 0 && second == 1) return 1;
    if (first == 1 && second == 0) return 2;
    if (first == 0 && second == 2) return 3;
    if (first == 1 && second == 2) return 4;
    if (first == 2 && second == 0) return 5;
    return 6; /* first == 2 && second == 1 */
}

static int64_t sat_add(int64_t x, int64_t d)
{
    if (d > 0 && x > INT64_MAX - d) return INT64_MAX;
    return x + d;
}

static int key_less(const edge_t *p, const edge_t *q)
{
    return p->t < q->t || (p->t == q->t && p->idx < q->idx);
}

static int cmp_key(const void *x, const void *y)
{
    const edge_t *p = *(const edge_t *const *)x, *q = *(const edge_t *const *)y;
    if (key_less(p, q)) return -1;
    if (key_less(q, p)) return 1;
    return 0;
}

/* number of edges of the key-sorted run [lo, hi) with key <= key(x) */
static uint64_t count_key_le(const edge_t *e, uint64_t lo, uint64_t hi, const edge_t *x)
{
    uint64_t b = lo, c = hi;
    while (b < c) {
        uint64_t mid = (b + c) / 2;
        if (!key_less(x, &e[mid])) b = mid + 1; else c = mid;
    }
    return b - lo;
}

/* number of edges of the run [lo, hi) with t <= lim */
static uint64_t count_t_le(const edge_t *e, uint64_t lo, uint64_t hi, int64_t lim)
{
    uint64_t b = lo, c = hi;
    while (b < c) {
        uint64_t mid = (b + c) / 2;
        if (e[mid].t <= lim) b = mid + 1; else c = mid;
    }
    return b - lo;
}

typedef struct {
    __int128 types[8];
    __int128 cells[48];
} acc_t;

/* Count the temporal triangles of static triangle {x, y, z} (pairs pxy, pxz, pyz). */
static void count_triangle(const graph_t *g, uint32_t x, uint32_t y, uint32_t z,
                           uint64_t pxy, uint64_t pxz, uint64_t pyz,
                           int64_t d13, int64_t d12, int64_t d23,
                           const edge_t **buf, acc_t *acc)
{
    /* name the vertices u < v < w by id; pair slots 0 = uv, 1 = uw, 2 = vw */
    uint32_t vs[3] = {x, y, z};
    for (int i = 0; i < 3; i++)
        for (int j = i + 1; j < 3; j++)
            if (vs[j] < vs[i]) { uint32_t tmp = vs[i]; vs[i] = vs[j]; vs[j] = tmp; }
    uint32_t u = vs[0], v = vs[1], w = vs[2];
    uint64_t pid[3] = {0, 0, 0};
    uint64_t cand[3] = {pxy, pxz, pyz};
    for (int i = 0; i < 3; i++) {
        uint64_t q = cand[i];
        if (g->pa[q] == u && g->pb[q] == v) pid[0] = q;
        else if (g->pa[q] == u && g->pb[q] == w) pid[1] = q;
        else pid[2] = q;
    }
    uint64_t L = 0;
    for (int s = 0; s < 3; s++)
        for (uint64_t i = g->pbeg[2 * pid[s]]; i < g->pbeg[2 * pid[s] + 2]; i++) buf[L++] = &g->e[i];
    qsort(buf, L, sizeof(const edge_t *), cmp_key);

    for (uint64_t i = 0; i < L; i++) {
        const edge_t *e1 = buf[i];
        for (uint64_t j = i + 1; j < L; j++) {
            const edge_t *e2 = buf[j];
            if ((__int128)e2->t - e1->t > d12) break;
            if (e2->a == e1->a && e2->b == e1->b) continue;
            /* slots of e1's and e2's pairs; the third slot is 3 - s1 - s2 */
            int s1 = (e1->a == u && e1->b == v) ? 0 : (e1->a == u ? 1 : 2);
            int s2 = (e2->a == u && e2->b == v) ? 0 : (e2->a == u ? 1 : 2);
            int s3 = 3 - s1 - s2;
            uint64_t p3 = pid[s3];
            int64_t lim = sat_add(e2->t, d23);
            int64_t lim2 = sat_add(e1->t, d13);
            if (lim2 < lim) lim = lim2;
            uint32_t a1 = e1->dir ? e1->b : e1->a, b1 = e1->dir ? e1->a : e1->b;
            uint32_t a2 = e2->dir ? e2->b : e2->a, b2 = e2->dir ? e2->a : e2->b;
            for (int d = 0; d < 2; d++) {
                uint64_t lo = g->pbeg[2 * p3 + d], hi = g->pbeg[2 * p3 + d + 1];
                if (lo == hi) continue;
                uint64_t after_e2 = count_key_le(g->e, lo, hi, e2);
                uint64_t within = count_t_le(g->e, lo, hi, lim);
                if (within <= after_e2) continue;
                uint64_t c = within - after_e2;
                uint32_t a3 = d ? g->pb[p3] : g->pa[p3], b3 = d ? g->pa[p3] : g->pb[p3];
                int ty = classify(a1, b1, a2, b2, a3, b3);
                acc->types[ty - 1] += c;
                /* cell: orientation from each pair's direction in this triple */
                int fwd[3];
                fwd[s1] = e1->dir == 0;
                fwd[s2] = e2->dir == 0;
                fwd[s3] = d == 0;
                int pi = pi_index(s1, s2);
                int rho = rho_index(fwd[0], fwd[1], fwd[2]);
                acc->cells[(pi - 1) * 8 + (rho - 1)] += c;
            }
        }
    }
}

typedef void (*tri_fn)(const graph_t *g, uint32_t x, uint32_t y, uint32_t z,
                       uint64_t pxy, uint64_t pxz, uint64_t pyz, void *ctx, int tid);

/* Every static triangle once, from its first vertex in (degree, id) order; in parallel over x. */
static void for_each_triangle(const graph_t *g, tri_fn fn, void *ctx, int nthreads)
{
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
    for (int64_t xi = 0; xi < (int64_t)g->n; xi++) {
        uint32_t x = (uint32_t)xi;
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        for (uint64_t i = g->adj_off[x]; i < g->adj_off[x + 1]; i++) {
            uint32_t y = g->adj_nbr[i];
            if (!before(g, x, y)) continue;
            for (uint64_t j = i + 1; j < g->adj_off[x + 1]; j++) {
                uint32_t z = g->adj_nbr[j];
                if (!before(g, x, z)) continue;
                int64_t q = find_pair(g, y, z);
                if (q < 0) continue;
                fn(g, x, y, z, g->adj_pair[i], g->adj_pair[j], (uint64_t)q, ctx, tid);
            }
        }
    }
}

typedef struct {
    int64_t d13, d12, d23;
    acc_t *acc;             /* one per thread */
    const edge_t ***buf;    /* one merge buffer per thread */
} count_ctx;

static void count_cb(const graph_t *g, uint32_t x, uint32_t y, uint32_t z,
                     uint64_t pxy, uint64_t pxz, uint64_t pyz, void *vctx, int tid)
{
    count_ctx *c = (count_ctx *)vctx;
    count_triangle(g, x, y, z, pxy, pxz, pyz, c->d13, c->d12, c->d23, c->buf[tid], &c->acc[tid]);
}

static int nthreads_of(int req)
{
#ifdef _OPENMP
    return req > 0 ? req : omp_get_max_threads();
#else
    (void)req;
    return 1;
#endif
}

/*
 * Per-type (types[k] = count of type T(k+1), Figure 2) and per-cell (cells[(pi-1)*8 + (rho-1)],
 * Figures 3 and 4, vertices named u < v < w by id) counts of (d13, d12, d23)-temporal triangles
 * among the edges with t_lo <= t <= t_hi.  Deltas are used as given (no rewriting); a delta of
 * INT64_MAX acts as infinity.  nthreads <= 0 uses the OpenMP default.  Returns 0, OR_EINVAL for a
 * node id >= n, a negative delta or t_lo > t_hi, OR_ENOMEM, or OR_EOVERFLOW when a total does not
 * fit in int64.  Either output pointer may be NULL.
 */
int oracle_count(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const int64_t *t,
                 int64_t d13, int64_t d12, int64_t d23, int64_t t_lo, int64_t t_hi, int nthreads,
                 int64_t types[8], int64_t cells[48])
{
    if (d13 < 0 || d12 < 0 || d23 < 0 || t_lo > t_hi) return OR_EINVAL;
    graph_t g;
    int rc = graph_build(&g, n, m, src, dst, t, t_lo, t_hi);
    if (rc) { graph_free(&g); return rc; }
    int nt = nthreads_of(nthreads);
    /* the largest per-triangle merge buffer: sum of the three largest pair sizes is enough, but
       a buffer of the kept edge count per thread is plain and always sufficient */
    uint64_t maxpair = 0;
    for (uint64_t q = 0; q < g.P; q++) {
        uint64_t s = g.pbeg[2 * q + 2] - g.pbeg[2 * q];
        if (s > maxpair) maxpair = s;
    }
    count_ctx c = {d13, d12, d23, NULL, NULL};
    c.acc = (acc_t *)calloc((size_t)nt, sizeof(acc_t));
    c.buf = (const edge_t ***)calloc((size_t)nt, sizeof(const edge_t **));
    if (!c.acc || !c.buf) { graph_free(&g); free(c.acc); free(c.buf); return OR_ENOMEM; }
    for (int i = 0; i < nt; i++) {
        c.buf[i] = (const edge_t **)malloc(sizeof(const edge_t *) * (3 * maxpair + 1));
        if (!c.buf[i]) rc = OR_ENOMEM;
    }
    if (!rc) for_each_triangle(&g, count_cb, &c, nt);
    __int128 ty[8] = {0}, ce[48] = {0};
    for (int i = 0; i < nt; i++) {
        for (int k = 0; k < 8; k++) ty[k] += c.acc[i].types[k];
        for (int k = 0; k < 48; k++) ce[k] += c.acc[i].cells[k];
        free(c.buf[i]);
    }
    free(c.acc); free(c.buf);
    graph_free(&g);
    if (rc) return rc;
    for (int k = 0; k < 8; k++) if (ty[k] > INT64_MAX) return OR_EOVERFLOW;
    for (int k = 0; k < 48; k++) if (ce[k] > INT64_MAX) return OR_EOVERFLOW;
    if (types) for (int k = 0; k < 8; k++) types[k] = (int64_t)ty[k];
    if (cells) for (int k = 0; k < 48; k++) cells[k] = (int64_t)ce[k];
    return OR_OK;
}

typedef struct {
    uint64_t *tri_count;      /* per thread */
    unsigned __int128 *sum3;  /* per thread */
    uint32_t *out;            /* NULL or 3 * cap ids, filled under a critical section */
    uint64_t cap, filled;
} tri_ctx;

static void tri_cb(const graph_t *g, uint32_t x, uint32_t y, uint32_t z,
                   uint64_t pxy, uint64_t pxz, uint64_t pyz, void *vctx, int tid)
{
    tri_ctx *c = (tri_ctx *)vctx;
    c->tri_count[tid]++;
    unsigned __int128 s = (unsigned __int128)(g->pbeg[2 * pxy + 2] - g->pbeg[2 * pxy]) *
                          (g->pbeg[2 * pxz + 2] - g->pbeg[2 * pxz]) *
                          (g->pbeg[2 * pyz + 2] - g->pbeg[2 * pyz]);
    c->sum3[tid] += s;
    if (c->out) {
        uint32_t vs[3] = {x, y, z};
        for (int i = 0; i < 3; i++)
            for (int j = i + 1; j < 3; j++)
                if (vs[j] < vs[i]) { uint32_t tmp = vs[i]; vs[i] = vs[j]; vs[j] = tmp; }
#pragma omp critical(oracle_tri_out)
        {
            if (c->filled < c->cap) {
                c->out[3 * c->filled] = vs[0];
                c->out[3 * c->filled + 1] = vs[1];
                c->out[3 * c->filled + 2] = vs[2];
            }
            c->filled++;
        }
    }
}

static int cmp_tri(const void *x, const void *y)
{
    const uint32_t *p = (const uint32_t *)x, *q = (const uint32_t *)y;
    for (int i = 0; i < 3; i++)
        if (p[i] != q[i]) return p[i] < q[i] ? -1 : 1;
    return 0;
}

/* Smallest-last removal with bucket queues (Matula & Beck; Batagelj & Zaversnik's form).
   core[v] = the largest k such that v belongs to the k-core; returns the degeneracy. */
static uint32_t core_numbers(const graph_t *g, uint32_t *core)
{
    uint32_t n = g->n;
    if (n == 0) return 0;
    uint32_t *deg = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *vert = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t md = 0;
    for (uint32_t v = 0; v < n; v++) {
        deg[v] = (uint32_t)(g->adj_off[v + 1] - g->adj_off[v]);
        if (deg[v] > md) md = deg[v];
    }
    uint32_t *bin = (uint32_t *)calloc((size_t)md + 2, sizeof(uint32_t));
    for (uint32_t v = 0; v < n; v++) bin[deg[v]]++;
    uint32_t start = 0;
    for (uint32_t d = 0; d <= md; d++) { uint32_t num = bin[d]; bin[d] = start; start += num; }
    for (uint32_t v = 0; v < n; v++) { pos[v] = bin[deg[v]]; vert[pos[v]] = v; bin[deg[v]]++; }
    for (uint32_t d = md; d >= 1; d--) bin[d] = bin[d - 1];
    bin[0] = 0;
    uint32_t kappa = 0;
    for (uint32_t i = 0; i < n; i++) {
        uint32_t v = vert[i];
        if (deg[v] > kappa) kappa = deg[v];
        for (uint64_t j = g->adj_off[v]; j < g->adj_off[v + 1]; j++) {
            uint32_t x = g->adj_nbr[j];
            if (deg[x] > deg[v]) {
                uint32_t dx = deg[x], px = pos[x], pw = bin[dx], w = vert[pw];
                if (x != w) { pos[x] = pw; vert[px] = w; pos[w] = px; vert[pw] = x; }
                bin[dx]++;
                deg[x]--;
            }
        }
    }
    for (uint32_t v = 0; v < n; v++) if (core) core[v] = deg[v];
    free(deg); free(vert); free(pos); free(bin);
    return kappa;
}

/*
 * Graph statistics of the edges with t_lo <= t <= t_hi (Table 1's columns): n, m (input edges),
 * self-loops dropped, edges kept in the window, static pairs, static triangles, degeneracy,
 * largest pair multiplicity (both directions), t_min/t_max of kept edges (INT64_MAX/INT64_MIN when
 * none), and the sum over static triangles of the product of the three pair multiplicities.
 * `core` (n entries, may be NULL) receives every vertex's core number.
 */
int oracle_stats_compute(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst,
                         const int64_t *t, int64_t t_lo, int64_t t_hi, int nthreads,
                         oracle_stats *st, uint32_t *core)
{
    if (t_lo > t_hi || !st) return OR_EINVAL;
    graph_t g;
    int rc = graph_build(&g, n, m, src, dst, t, t_lo, t_hi);
    if (rc) { graph_free(&g); return rc; }
    memset(st, 0, sizeof(*st));
    st->n = n;
    st->m = m;
    st->self_loops = g.self_loops;
    st->m_window = g.m;
    st->m_static = g.P;
    st->t_min = g.t_min;
    st->t_max = g.t_max;
    for (uint64_t q = 0; q < g.P; q++) {
        uint64_t s = g.pbeg[2 * q + 2] - g.pbeg[2 * q];
        if (s > st->max_multiplicity) st->max_multiplicity = (uint32_t)s;
    }
    st->degeneracy = core_numbers(&g, core);
    int nt = nthreads_of(nthreads);
    tri_ctx c = {0};
    c.tri_count = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
    c.sum3 = (unsigned __int128 *)calloc((size_t)nt, sizeof(unsigned __int128));
    if (!c.tri_count || !c.sum3) { graph_free(&g); free(c.tri_count); free(c.sum3); return OR_ENOMEM; }
    for_each_triangle(&g, tri_cb, &c, nt);
    unsigned __int128 s3 = 0;
    for (int i = 0; i < nt; i++) { st->n_triangles += c.tri_count[i]; s3 += c.sum3[i]; }
    st->sum_sigma3_lo = (uint64_t)s3;
    st->sum_sigma3_hi = (uint64_t)(s3 >> 64);
    free(c.tri_count); free(c.sum3);
    graph_free(&g);
    return OR_OK;
}

/*
 * The static triangles of the edges with t_lo <= t <= t_hi as node-id triples (a < b < c) in
 * lexicographic order.  Writes min(count, cap) triples to out (3 ids each) and returns the count,
 * or a negative error code.
 */
int64_t oracle_triangles(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst,
                         const int64_t *t, int64_t t_lo, int64_t t_hi, uint32_t *out, uint64_t cap)
{
    if (t_lo > t_hi) return OR_EINVAL;
    graph_t g;
    int rc = graph_build(&g, n, m, src, dst, t, t_lo, t_hi);
    if (rc) { graph_free(&g); return rc; }
    tri_ctx c = {0};
    uint64_t one = 0;
    unsigned __int128 s3 = 0;
    c.tri_count = &one;
    c.sum3 = &s3;
    c.out = out;
    c.cap = out ? cap : 0;
    for_each_triangle(&g, tri_cb, &c, 1);
    if (out) qsort(out, c.filled < cap ? c.filled : cap, 3 * sizeof(uint32_t), cmp_tri);
    graph_free(&g);
    return (int64_t)one;
}
