/*
 * CPU DOTTT: the paper's own method, sequential, as a second CPU baseline and as an independent
 * cross-check of its algorithms against the plain oracle (dottt_oracle.c).
 *
 * TEST AND BASELINE INFRASTRUCTURE ONLY.  The test-suite and the benchmark's CPU-baseline leg are
 * its only callers; it shares no code with the oracle or with the GPU library.
 *
 * The steps follow the paper's top-level procedure (Algorithm 4, Section 5):
 *   1. extract the static graph G of the (windowed) temporal graph and group its temporal edges
 *      by pair and direction, each group sorted by (timestamp, input position);
 *   2. the degeneracy ordering of G by repeatedly removing a vertex of minimum remaining degree
 *      (Section 3; the bucket-queue form of Matula and Beck, linear time);
 *   3. orient G along the ordering (the DAG G_prec) and list every static triangle <u, v, w>,
 *      u < v < w in the ordering, by marking N+(u) and scanning N+(v) for each v in N+(u)
 *      (Section 5);
 *   4. for every triangle, every temporal ordering pi (Figure 3) and orientation rho (Figure 4),
 *      count the temporal triangles by the prefix-count procedures -- Algorithm 1 when {v,w} is
 *      third in pi, the Appendix procedures when it is second or first -- and add the count to
 *      type psi(pi, rho) (Table 2).
 *
 * Readings of the paper used here (the same ones the rest of the repository uses):
 *  - edges are totally ordered by key (t, input position); order constraints use keys and the
 *    delta constraints use timestamps, which is Definition 1 when timestamps are distinct;
 *  - deltas are normalised first: d12 <- min(d12, d13), d23 <- min(d23, d13),
 *    d13 <- min(d13, d12 + d23) (the same constraint set; the procedures' index inequalities
 *    need it), and clamped to the time span;
 *  - the window [t_lo, t_hi] is inclusive and means counting the graph filtered to it;
 *  - self-loops lie on no triangle and are dropped.
 * The procedures are restated for keys, so equal timestamps are counted once in the key order:
 *  - {v,w} third (Algorithm 1; pi1, pi2): for e2 in S2, the e1 in S1 with key < k2 and
 *    t1 >= t2 - d12 form an index range [a, b); those with t1 <= t2 - d13 + d23 (a prefix [a, c))
 *    take e3 up to t1 + d13, the rest up to t2 + d23, always with key > k2.  A prefix sum over S1
 *    of "edges of S3 up to t1 + d13" gives the first part in O(1).
 *  - {v,w} second (pi3, pi4): for e1 in S1, the e3 in S3 with key > k1 and t3 <= t1 + d13 split
 *    at t1 + min(d12, d23) and t1 + max(d12, d23); in each part the e2 of S2 between them are a
 *    difference of two prefix sums over S3 (of "S2 keys below k3" and "S2 times below t3 - d23")
 *    or a constant.
 *  - {v,w} first (pi5, pi6): for e2 in S2, the e3 in S3 with key > k2 and t3 <= t2 + d23 split at
 *    t2 + d13 - d12; before it every e1 from t2 - d12 on qualifies, after it those from t3 - d13
 *    on (a prefix sum over S3 of "S1 times below t3 - d13").
 * Only the lists on the two pairs at the source vertex u are walked; {v,w} is only searched.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

typedef struct {
    int64_t t;
    uint64_t i;   /* input position */
} Key;

static int key_less(Key a, Key b) { return a.t < b.t || (a.t == b.t && a.i < b.i); }

/* number of entries of s[0, n) with key < k */
static int64_t cnt_key_lt(const Key *s, int64_t n, Key k) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (key_less(s[mid], k)) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* number of entries with timestamp <= x */
static int64_t cnt_t_le(const Key *s, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (s[mid].t <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* number of entries with timestamp < x */
static int64_t cnt_t_lt(const Key *s, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (s[mid].t < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int64_t clamp64(int64_t x, int64_t lo, int64_t hi) { return x < lo ? lo : (x > hi ? hi : x); }

typedef struct {
    const Key *s;
    int64_t n;
} List;

typedef struct {
    int64_t d13, d12, d23;
    int64_t *pa, *pb;   /* prefix scratch, max list length + 1 each */
} Ctx;

/* {v,w} third (pi1, pi2) */
static int64_t vw_third(const Ctx *c, List S1, List S2, List S3) {
    if (!S1.n || !S2.n || !S3.n) return 0;
    int64_t *pe = c->pa;   /* pe[r] = sum over S1[0, r) of #S3 with t <= t1 + d13 */
    pe[0] = 0;
    for (int64_t r = 0; r < S1.n; ++r) pe[r + 1] = pe[r] + cnt_t_le(S3.s, S3.n, S1.s[r].t + c->d13);
    int64_t total = 0;
    for (int64_t j = 0; j < S2.n; ++j) {
        const Key e2 = S2.s[j];
        const int64_t a = cnt_t_lt(S1.s, S1.n, e2.t - c->d12), b = cnt_key_lt(S1.s, S1.n, e2);
        if (b <= a) continue;
        const int64_t m = clamp64(cnt_t_le(S1.s, S1.n, e2.t - c->d13 + c->d23), a, b);
        const int64_t after = cnt_key_lt(S3.s, S3.n, e2);   /* S3 entries with key < k2 */
        total += (pe[m] - pe[a]) - (m - a) * after;
        total += (b - m) * (cnt_t_le(S3.s, S3.n, e2.t + c->d23) - after);
    }
    return total;
}

/* {v,w} second (pi3, pi4) */
static int64_t vw_second(const Ctx *c, List S1, List S2, List S3) {
    if (!S1.n || !S2.n || !S3.n) return 0;
    int64_t *pA = c->pa, *pB = c->pb;   /* over S3: #S2 with key < k3; #S2 with t < t3 - d23 */
    pA[0] = pB[0] = 0;
    for (int64_t r = 0; r < S3.n; ++r) {
        pA[r + 1] = pA[r] + cnt_key_lt(S2.s, S2.n, S3.s[r]);
        pB[r + 1] = pB[r] + cnt_t_lt(S2.s, S2.n, S3.s[r].t - c->d23);
    }
    const int64_t lo = c->d12 < c->d23 ? c->d12 : c->d23, hi = c->d12 < c->d23 ? c->d23 : c->d12;
    int64_t total = 0;
    for (int64_t j = 0; j < S1.n; ++j) {
        const Key e1 = S1.s[j];
        const int64_t f = cnt_key_lt(S3.s, S3.n, e1);
        int64_t x1 = cnt_t_le(S3.s, S3.n, e1.t + lo);
        x1 = x1 > f ? x1 : f;
        int64_t x2 = cnt_t_le(S3.s, S3.n, e1.t + hi);
        x2 = x2 > x1 ? x2 : x1;
        int64_t x3 = cnt_t_le(S3.s, S3.n, e1.t + c->d13);
        x3 = x3 > x2 ? x3 : x2;
        const int64_t below = cnt_key_lt(S2.s, S2.n, e1), upto = cnt_t_le(S2.s, S2.n, e1.t + c->d12);
        /* t3 <= t1 + min(d12, d23): every e2 between e1 and e3 in key order */
        total += (pA[x1] - pA[f]) - (x1 - f) * below;
        /* between the two: bounded by t1 + d12 (d12 <= d23) or by t3 - d23 (d23 < d12) */
        if (c->d12 <= c->d23) total += (x2 - x1) * (upto - below);
        else total += (pA[x2] - pA[x1]) - (pB[x2] - pB[x1]);
        /* beyond both: from t3 - d23 up to t1 + d12 */
        total += (x3 - x2) * upto - (pB[x3] - pB[x2]);
    }
    return total;
}

/* {v,w} first (pi5, pi6) */
static int64_t vw_first(const Ctx *c, List S1, List S2, List S3) {
    if (!S1.n || !S2.n || !S3.n) return 0;
    int64_t *pC = c->pa;   /* over S3: #S1 with t < t3 - d13 */
    pC[0] = 0;
    for (int64_t r = 0; r < S3.n; ++r) pC[r + 1] = pC[r] + cnt_t_lt(S1.s, S1.n, S3.s[r].t - c->d13);
    int64_t total = 0;
    for (int64_t j = 0; j < S2.n; ++j) {
        const Key e2 = S2.s[j];
        const int64_t f = cnt_key_lt(S3.s, S3.n, e2);
        int64_t sp = cnt_t_le(S3.s, S3.n, e2.t + c->d13 - c->d12);
        sp = sp > f ? sp : f;
        int64_t e = cnt_t_le(S3.s, S3.n, e2.t + c->d23);
        e = e > sp ? e : sp;
        const int64_t before = cnt_key_lt(S1.s, S1.n, e2);
        total += (sp - f) * (before - cnt_t_lt(S1.s, S1.n, e2.t - c->d12));
        total += (e - sp) * before - (pC[e] - pC[sp]);
    }
    return total;
}

/* Figure 4: for orientation rho (1..8), whether each pair points away from its vertex that comes
 * first in u, v, w: uv (u->v), uw (u->w), vw (v->w) */
static const int kRhoFwd[8][3] = {
    {1, 1, 1}, {1, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {0, 0, 0}, {0, 1, 0}, {0, 0, 1},
};
/* Figure 3: pairs of pi (1..6) in time order; 0 = uv, 1 = uw, 2 = vw */
static const int kPi[6][3] = {{0, 1, 2}, {1, 0, 2}, {0, 2, 1}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
/* Table 2: type of (pi, rho) */
static const int kPsi[6][8] = {
    {7, 6, 5, 8, 3, 2, 4, 1}, {5, 3, 7, 4, 6, 1, 8, 2}, {3, 2, 1, 4, 7, 6, 8, 5},
    {1, 7, 3, 8, 2, 5, 4, 6}, {6, 1, 2, 8, 5, 3, 4, 7}, {2, 5, 6, 4, 1, 7, 8, 3},
};

typedef struct {
    uint64_t key;   /* pair (a, b), a < b by id, as a * n + b */
    int dir;        /* 0: a -> b */
    Key k;
} Rec;

static int rec_cmp(const void *x, const void *y) {
    const Rec *a = (const Rec *)x, *b = (const Rec *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->dir != b->dir) return a->dir < b->dir ? -1 : 1;
    if (key_less(a->k, b->k)) return -1;
    if (key_less(b->k, a->k)) return 1;
    return 0;
}

/*
 * Counts per type into out[8] (out[i] = type i + 1).  Returns 0, -22 for invalid arguments or
 * -12 when memory runs out.  *seconds (optional): time of steps 2-4 (after the extraction).
 */
int cpu_dottt_count(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const int64_t *t,
                    int64_t d13, int64_t d12, int64_t d23, int64_t t_lo, int64_t t_hi, int64_t *out,
                    double *seconds) {
    for (int i = 0; i < 8; ++i) out[i] = 0;
    if (seconds) *seconds = 0.0;
    if (d13 < 0 || d12 < 0 || d23 < 0 || t_lo > t_hi) return -22;
    for (uint64_t e = 0; e < m; ++e)
        if (src[e] >= n || dst[e] >= n) return -22;
    /* 1. extraction: kept edges grouped by pair, then direction, then key */
    uint64_t mk = 0;
    for (uint64_t e = 0; e < m; ++e) mk += (src[e] != dst[e] && t[e] >= t_lo && t[e] <= t_hi);
    if (mk == 0) return 0;
    Rec *rec = (Rec *)malloc(mk * sizeof(Rec));
    if (!rec) return -12;
    int64_t tmin = INT64_MAX, tmax = INT64_MIN;
    uint64_t j = 0;
    for (uint64_t e = 0; e < m; ++e) {
        if (src[e] == dst[e] || t[e] < t_lo || t[e] > t_hi) continue;
        const uint32_t a = src[e] < dst[e] ? src[e] : dst[e], b = src[e] < dst[e] ? dst[e] : src[e];
        rec[j].key = (uint64_t)a * n + b;
        rec[j].dir = src[e] == a ? 0 : 1;
        rec[j].k.t = t[e];
        rec[j].k.i = e;
        tmin = t[e] < tmin ? t[e] : tmin;
        tmax = t[e] > tmax ? t[e] : tmax;
        ++j;
    }
    qsort(rec, mk, sizeof(Rec), rec_cmp);
    const int64_t span = tmax - tmin;
    d13 = d13 > span ? span : d13;
    d12 = d12 > span ? span : d12;
    d23 = d23 > span ? span : d23;
    d12 = d12 < d13 ? d12 : d13;
    d23 = d23 < d13 ? d23 : d13;
    d13 = d13 < d12 + d23 ? d13 : d12 + d23;

    struct timespec ts0, ts1;
    clock_gettime(CLOCK_MONOTONIC, &ts0);
    /* pairs and their three offsets: direction a -> b in [off[3p], off[3p+1]), b -> a up to off[3p+2] */
    uint64_t np = 0;
    for (uint64_t e = 0; e < mk; ++e) np += (e == 0 || rec[e].key != rec[e - 1].key);
    Key *keys = (Key *)malloc(mk * sizeof(Key));
    uint64_t *off = (uint64_t *)malloc((3 * np + 1) * sizeof(uint64_t));
    uint32_t *pa = (uint32_t *)malloc(np * sizeof(uint32_t)), *pb = (uint32_t *)malloc(np * sizeof(uint32_t));
    uint64_t *deg0 = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    int rc = 0;
    if (!keys || !off || !pa || !pb || !deg0) { rc = -12; goto done0; }
    {
        uint64_t p = 0, maxs = 0;
        for (uint64_t e = 0; e < mk;) {
            uint64_t f = e;
            while (f < mk && rec[f].key == rec[e].key) ++f;
            uint64_t mid = e;
            while (mid < f && rec[mid].dir == 0) ++mid;
            off[3 * p] = e;
            off[3 * p + 1] = mid;
            off[3 * p + 2] = f;
            pa[p] = (uint32_t)(rec[e].key / n);
            pb[p] = (uint32_t)(rec[e].key % n);
            for (uint64_t x = e; x < f; ++x) keys[x] = rec[x].k;
            maxs = f - e > maxs ? f - e : maxs;
            ++deg0[pa[p]];
            ++deg0[pb[p]];
            ++p;
            e = f;
        }
        free(rec);
        rec = NULL;
        /* undirected CSR of G */
        uint64_t *row = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
        uint32_t *nb = (uint32_t *)malloc(2 * np * sizeof(uint32_t));
        uint64_t *nbp = (uint64_t *)malloc(2 * np * sizeof(uint64_t));
        uint64_t *fill = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
        uint32_t *deg = (uint32_t *)malloc(((size_t)n + 1) * sizeof(uint32_t));
        uint32_t *order = (uint32_t *)malloc(((size_t)n + 1) * sizeof(uint32_t));
        uint32_t *pos = (uint32_t *)malloc(((size_t)n + 1) * sizeof(uint32_t));
        uint32_t *bin = NULL;
        uint64_t *orow = NULL, *ocnt = NULL;
        uint32_t *onb = NULL, *stamp = NULL;
        uint64_t *onbp = NULL, *mark = NULL;
        int64_t *scratch = NULL;
        if (!row || !nb || !nbp || !fill || !deg || !order || !pos) { rc = -12; goto done1; }
        row[0] = 0;
        for (uint32_t v = 0; v < n; ++v) row[v + 1] = row[v] + deg0[v];
        memcpy(fill, row, ((size_t)n + 1) * sizeof(uint64_t));
        for (uint64_t q = 0; q < np; ++q) {
            nb[fill[pa[q]]] = pb[q];
            nbp[fill[pa[q]]++] = q;
            nb[fill[pb[q]]] = pa[q];
            nbp[fill[pb[q]]++] = q;
        }
        /* 2. degeneracy ordering: vertices kept in an array sorted by current degree, with the
         * start of every degree's block; removing the first vertex of minimum degree lowers each
         * remaining neighbour's degree by swapping it to the front of its block */
        uint32_t maxd = 0;
        for (uint32_t v = 0; v < n; ++v) {
            deg[v] = (uint32_t)deg0[v];
            maxd = deg[v] > maxd ? deg[v] : maxd;
        }
        bin = (uint32_t *)calloc((size_t)maxd + 2, sizeof(uint32_t));
        if (!bin) { rc = -12; goto done1; }
        for (uint32_t v = 0; v < n; ++v) ++bin[deg[v]];
        {
            uint32_t start = 0;
            for (uint32_t d = 0; d <= maxd; ++d) {
                const uint32_t c = bin[d];
                bin[d] = start;
                start += c;
            }
        }
        for (uint32_t v = 0; v < n; ++v) {
            pos[v] = bin[deg[v]]++;
            order[pos[v]] = v;
        }
        for (uint32_t d = maxd; d > 0; --d) bin[d] = bin[d - 1];
        bin[0] = 0;
        for (uint32_t i = 0; i < n; ++i) {
            const uint32_t v = order[i];   /* removed now: rank i */
            for (uint64_t x = row[v]; x < row[v + 1]; ++x) {
                const uint32_t w = nb[x];
                if (pos[w] <= i || deg[w] <= deg[v]) continue;   /* removed, or already minimal */
                const uint32_t dw = deg[w], pw = pos[w], first = bin[dw] > i + 1 ? bin[dw] : i + 1;
                const uint32_t y = order[first];
                if (y != w) {
                    order[pw] = y;
                    pos[y] = pw;
                    order[first] = w;
                    pos[w] = first;
                }
                bin[dw] = first + 1;
                --deg[w];
            }
        }
        /* pos[v] is now v's rank.  3. G_prec: N+(v) = neighbours of higher rank */
        orow = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
        ocnt = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
        onb = (uint32_t *)malloc((np + 1) * sizeof(uint32_t));
        onbp = (uint64_t *)malloc((np + 1) * sizeof(uint64_t));
        stamp = (uint32_t *)malloc(((size_t)n + 1) * sizeof(uint32_t));
        mark = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
        scratch = (int64_t *)malloc(2 * (maxs + 1) * sizeof(int64_t));
        if (!orow || !ocnt || !onb || !onbp || !stamp || !mark || !scratch) { rc = -12; goto done1; }
        for (uint64_t q = 0; q < np; ++q) ++ocnt[pos[pa[q]] < pos[pb[q]] ? pa[q] : pb[q]];
        orow[0] = 0;
        for (uint32_t v = 0; v < n; ++v) orow[v + 1] = orow[v] + ocnt[v];
        memcpy(ocnt, orow, (size_t)n * sizeof(uint64_t));
        for (uint64_t q = 0; q < np; ++q) {
            const int a_first = pos[pa[q]] < pos[pb[q]];
            const uint32_t tail = a_first ? pa[q] : pb[q], head = a_first ? pb[q] : pa[q];
            onb[ocnt[tail]] = head;
            onbp[ocnt[tail]++] = q;
        }
        for (uint32_t v = 0; v < n; ++v) stamp[v] = 0xffffffffu;
        Ctx c = {d13, d12, d23, scratch, scratch + maxs + 1};
        /* 4. every triangle <u, v, w>: mark N+(u), then for v in N+(u) look for w in N+(v) */
        for (uint32_t u = 0; u < n; ++u) {
            for (uint64_t x = orow[u]; x < orow[u + 1]; ++x) {
                stamp[onb[x]] = u;
                mark[onb[x]] = onbp[x];
            }
            for (uint64_t x = orow[u]; x < orow[u + 1]; ++x) {
                const uint32_t v = onb[x];
                const uint64_t p_uv = onbp[x];
                for (uint64_t y = orow[v]; y < orow[v + 1]; ++y) {
                    const uint32_t w = onb[y];
                    if (stamp[w] != u) continue;
                    const uint64_t pr[3] = {p_uv, mark[w], onbp[y]};
                    /* the first vertex of each pair in the naming u, v, w */
                    const uint32_t first[3] = {u, u, v};
                    for (int rho = 0; rho < 8; ++rho) {
                        List L[3];
                        for (int e = 0; e < 3; ++e) {
                            const uint64_t q = pr[e];
                            /* direction a -> b of pair q is "forward" when its first vertex is a */
                            const int fwd = kRhoFwd[rho][e];
                            const int ab = (pa[q] == first[e]) ? fwd : !fwd;
                            const uint64_t lo = ab ? off[3 * q] : off[3 * q + 1];
                            const uint64_t hi = ab ? off[3 * q + 1] : off[3 * q + 2];
                            L[e].s = keys + lo;
                            L[e].n = (int64_t)(hi - lo);
                        }
                        for (int pi = 0; pi < 6; ++pi) {
                            const List S1 = L[kPi[pi][0]], S2 = L[kPi[pi][1]], S3 = L[kPi[pi][2]];
                            int64_t cnt;
                            if (pi < 2) cnt = vw_third(&c, S1, S2, S3);
                            else if (pi < 4) cnt = vw_second(&c, S1, S2, S3);
                            else cnt = vw_first(&c, S1, S2, S3);
                            out[kPsi[pi][rho] - 1] += cnt;
                        }
                    }
                }
            }
        }
    done1:
        free(row); free(nb); free(nbp); free(fill); free(deg); free(order); free(pos); free(bin);
        free(orow); free(ocnt); free(onb); free(onbp); free(stamp); free(mark); free(scratch);
    }
done0:
    free(rec); free(keys); free(off); free(pa); free(pb); free(deg0);
    clock_gettime(CLOCK_MONOTONIC, &ts1);
    if (seconds) *seconds = (double)(ts1.tv_sec - ts0.tv_sec) + 1e-9 * (double)(ts1.tv_nsec - ts0.tv_nsec);
    if (rc) for (int i = 0; i < 8; ++i) out[i] = 0;
    return rc;
}
