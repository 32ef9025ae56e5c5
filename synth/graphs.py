"""Seeded generators for directed temporal multigraphs with heavy-tailed multiplicities.

Every graph is a list of directed temporal edges (src, dst, t) with uint32 node ids and int64
timestamps; the list order is the tie-break order for equal timestamps.  The generators stand in
for the SNAP / KONECT / Bitcoin datasets that the paper measures on (Section 6); none of those
datasets' records are reproduced here.

Static structure is a directed Chung-Lu graph: node weights w_i proportional to i^(-1/(gamma-1)),
capped at sqrt(sum w), randomly permuted (independently for out- and in-weights), and pairs
(u ~ w_out, v ~ w_in) drawn i.i.d. with self-pairs rejected and unordered duplicates dropped.
Each static pair carries a multiplicity of temporal edges whose directions and timestamps are
drawn per workload.  This module draws random numbers only; it counts nothing.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2106027620
EPOCH = 1_262_304_000          # 2010-01-01T00:00:00Z; base of the bursty workloads' clocks
YEAR = 31_557_600              # 365.25 days in seconds
SESSION_GAP = 300.0            # mean gap between edges of one burst (s)


@dataclass
class TemporalGraph:
    n: int
    src: np.ndarray            # uint32[m]
    dst: np.ndarray            # uint32[m]
    t: np.ndarray              # int64[m]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def arrays(self):
        return self.src, self.dst, self.t


# ----------------------------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------------------------

def _cl_cdf(rng, n: int, gamma: float, weight_sum: float) -> np.ndarray:
    """Cumulative sampling distribution of a permuted, capped Chung-Lu weight sequence."""
    i = np.arange(1, n + 1, dtype=np.float64)
    w = i ** (-1.0 / (gamma - 1.0))
    w *= weight_sum / w.sum()
    np.minimum(w, np.sqrt(weight_sum), out=w)
    wp = np.empty(n, dtype=np.float64)
    wp[rng.permutation(n)] = w
    cdf = np.cumsum(wp)
    cdf /= cdf[-1]
    return cdf


def _draw_nodes(rng, cdf: np.ndarray, k: int) -> np.ndarray:
    x = np.searchsorted(cdf, rng.random(k), side="right")
    np.minimum(x, cdf.shape[0] - 1, out=x)
    return x.astype(np.int64)


def _distinct_pairs(rng, n, cdf_out, cdf_in, target, prefix=None):
    """Distinct unordered pairs in first-occurrence order, each kept in its drawn orientation.

    `prefix` (u, v) pairs are placed first.  Returns (u, v) int64 arrays of length `target`.
    """
    if prefix is not None:
        pu, pv = prefix
    else:
        pu = np.empty(0, np.int64)
        pv = np.empty(0, np.int64)
    u_all, v_all = pu, pv
    have = 0
    while True:
        need = max(target - have, 0)
        k = int(need * 1.3) + 4096
        u = _draw_nodes(rng, cdf_out, k)
        v = _draw_nodes(rng, cdf_in, k)
        ok = u != v
        u_all = np.concatenate([u_all, u[ok]])
        v_all = np.concatenate([v_all, v[ok]])
        key = np.minimum(u_all, v_all) * n + np.maximum(u_all, v_all)
        _, first = np.unique(key, return_index=True)
        have = first.shape[0]
        if have >= target:
            first.sort()
            first = first[:target]
            return u_all[first], v_all[first]
        first.sort()
        u_all, v_all = u_all[first], v_all[first]


def _expand(rng, u, v, mult, p_keep):
    """Temporal edges of each static pair; each keeps the drawn orientation with prob p_keep."""
    pid = np.repeat(np.arange(u.shape[0], dtype=np.int64), mult)
    keep = rng.random(pid.shape[0]) < p_keep
    up, vp = u[pid], v[pid]
    src = np.where(keep, up, vp).astype(np.uint32)
    dst = np.where(keep, vp, up).astype(np.uint32)
    return pid, src, dst


def _bursty_times(rng, mult, span, anchors=None):
    """Bursty timestamps, one array aligned with np.repeat(arange(P), mult).

    A pair with multiplicity k has 1 + Binomial(k-1, 1/8) sessions whose starts are uniform over
    [0, span); each edge joins a uniformly chosen session and follows the previous edge of its
    session after an Exp(mean 300 s) gap.  `anchors` (pair index array, start array) re-anchors
    session 0 of those pairs.  Times are floored to whole seconds and clipped to [0, span).
    """
    P = mult.shape[0]
    m = int(mult.sum())
    S = 1 + rng.binomial(mult - 1, 1.0 / 8.0)
    base = np.zeros(P, dtype=np.int64)
    np.cumsum(S[:-1], out=base[1:])
    starts = rng.random(int(S.sum())) * span
    if anchors is not None:
        apair, astart = anchors
        starts[base[apair]] = astart
    pid = np.repeat(np.arange(P, dtype=np.int64), mult)
    sess = (rng.random(m) * S[pid]).astype(np.int64)
    np.minimum(sess, S[pid] - 1, out=sess)
    gsess = base[pid] + sess
    del sess
    order = np.argsort(gsess, kind="stable")
    gs = gsess[order]
    del gsess
    gaps = rng.exponential(SESSION_GAP, m)
    cs = np.cumsum(gaps)
    first = np.empty(m, dtype=bool)
    first[0] = True
    np.not_equal(gs[1:], gs[:-1], out=first[1:])
    gstart = np.where(first, np.arange(m, dtype=np.int64), 0)
    np.maximum.accumulate(gstart, out=gstart)
    off = cs - cs[gstart] + gaps[gstart]
    del cs, gaps, first, gstart
    ts = np.floor(starts[gs] + off)
    del off, gs
    t = np.empty(m, dtype=np.float64)
    t[order] = ts
    del ts, order
    np.clip(t, 0, span - 1, out=t)
    return t.astype(np.int64)


def _time_sorted(rng, src, dst, t):
    """Reorder the edge list by timestamp; equal timestamps keep a random relative order."""
    perm = rng.permutation(t.shape[0])
    order = perm[np.argsort(t[perm], kind="stable")]
    return src[order], dst[order], t[order]


def _planted_triangles(rng, cdf, count, span):
    """`count` vertex triples drawn by weight, as 3*count pairs plus one burst anchor per triple."""
    n = cdf.shape[0]
    x = _draw_nodes(rng, cdf, count)
    y = _draw_nodes(rng, cdf, count)
    z = _draw_nodes(rng, cdf, count)
    ok = (x != y) & (y != z) & (x != z)
    x, y, z = x[ok], y[ok], z[ok]
    anchor = rng.random(x.shape[0]) * span
    pu = np.stack([x, y, x], axis=1).reshape(-1)
    pv = np.stack([y, z, z], axis=1).reshape(-1)
    pa = np.repeat(anchor, 3)
    key = np.minimum(pu, pv) * n + np.maximum(pu, pv)
    _, first = np.unique(key, return_index=True)
    first.sort()
    return (pu[first], pv[first]), pa[first]


# ----------------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------------

def tiny_multigraph(seed: int, n: int = 6, m: int = 16, t_range: int = 12, p_pair: float = 0.7):
    """A small random directed multigraph for exhaustive checks, with many equal timestamps.

    Pairs of a random static graph on `n` nodes (each pair present with probability p_pair) are
    drawn uniformly per edge, in a random direction, with t uniform over {0..t_range-1}.  A few
    self-loops are mixed in so that dropping them is exercised.
    """
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p_pair
    if keep.sum() < 3:
        keep[:3] = True
    pu, pv = iu[keep], ju[keep]
    k = rng.integers(0, pu.shape[0], m)
    flip = rng.random(m) < 0.5
    src = np.where(flip, pv[k], pu[k]).astype(np.uint32)
    dst = np.where(flip, pu[k], pv[k]).astype(np.uint32)
    loops = rng.random(m) < 0.05
    dst = np.where(loops, src, dst).astype(np.uint32)
    t = rng.integers(0, t_range, m).astype(np.int64)
    return TemporalGraph(n, src, dst, t, name=f"tiny(seed={seed},n={n},m={m})")


def seed_graph(seed: int = SEED_BASE):
    """The 50-node, 300-temporal-edge graph that brute force over all edge triples can check.

    120 random static pairs on 50 nodes; 300 edges drawn uniformly over them in random directions
    with t uniform over {0..1999}, so that counts are dense and equal timestamps occur.
    """
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(50, 1)
    pick = rng.choice(iu.shape[0], 120, replace=False)
    pu, pv = iu[pick], ju[pick]
    k = rng.integers(0, 120, 300)
    flip = rng.random(300) < 0.5
    src = np.where(flip, pv[k], pu[k]).astype(np.uint32)
    dst = np.where(flip, pu[k], pv[k]).astype(np.uint32)
    t = rng.integers(0, 2000, 300).astype(np.int64)
    return TemporalGraph(50, src, dst, t, name="seed50x300")


def plain_tiny(seed: int = SEED_BASE + 0):
    """n=1,000, 5,000 static pairs (gamma=2.5), multiplicity 1+Geometric(1/2), t ~ U{0..10^6-1},
    uniformly random directions."""
    rng = np.random.default_rng(seed)
    n, ms = 1000, 5000
    co = _cl_cdf(rng, n, 2.5, 2.0 * ms)
    ci = _cl_cdf(rng, n, 2.5, 2.0 * ms)
    u, v = _distinct_pairs(rng, n, co, ci, ms)
    mult = rng.geometric(0.5, ms)
    _, src, dst = _expand(rng, u, v, mult, 0.5)
    t = rng.integers(0, 10**6, src.shape[0]).astype(np.int64)
    src, dst, t = _time_sorted(rng, src, dst, t)
    return TemporalGraph(n, src, dst, t, name="plain_tiny_n1k",
                         meta={"deltas": (3600, 3600, 3600)})


def _bursty_chung_lu(rng, n, gamma, ms_draw, mult_fn, span, m_target=None, planted_frac=0.01):
    co = _cl_cdf(rng, n, gamma, 2.0 * ms_draw)
    ci = _cl_cdf(rng, n, gamma, 2.0 * ms_draw)
    prefix, panchor = _planted_triangles(rng, co, int(planted_frac * ms_draw), span)
    u, v = _distinct_pairs(rng, n, co, ci, ms_draw, prefix=prefix)
    mult = mult_fn(rng, u.shape[0])
    if m_target is not None:
        cs = np.cumsum(mult)
        cut = int(np.searchsorted(cs, m_target, side="left")) + 1
        cut = min(cut, u.shape[0])
        u, v, mult = u[:cut], v[:cut], mult[:cut]
        excess = int(mult.sum()) - m_target
        if excess > 0:
            mult[-1] -= excess
    npl = panchor.shape[0]
    apair = np.arange(min(npl, u.shape[0]), dtype=np.int64)
    astart = panchor[: apair.shape[0]] + rng.exponential(SESSION_GAP, apair.shape[0])
    t = _bursty_times(rng, mult, span, anchors=(apair, astart))
    _, src, dst = _expand(rng, u, v, mult, 0.75)
    t += EPOCH
    src, dst, t = _time_sorted(rng, src, dst, t)
    return src, dst, t, int(u.shape[0])


def plain_medium(seed: int = SEED_BASE + 1):
    """n=10^6, gamma=2.1, multiplicity min(Zipf(2), 10^4), static pairs added until the temporal
    edges reach 10^7; bursty timestamps over 3 years; 1% of static pairs are planted triangles
    with a common burst."""
    rng = np.random.default_rng(seed)
    n = 10**6
    span = 3 * YEAR
    src, dst, t, ms = _bursty_chung_lu(
        rng, n, 2.1, 1_700_000,
        lambda r, k: np.minimum(r.zipf(2.0, k), 10**4).astype(np.int64),
        span, m_target=10**7)
    return TemporalGraph(n, src, dst, t, name="plain_medium_n1M_m10M",
                         meta={"deltas": (3600, 3600, 3600), "static_pairs_drawn": ms})


def plain_full(seed: int = SEED_BASE + 2, n: int = 2_600_000, ms: int = 36_000_000):
    """n=2.6M, 36M static pairs (gamma=2.0); multiplicity 1 with probability 0.9749, otherwise
    min(Zipf(1.8), 10^5) (about 63M temporal edges with a heavy multi-edge tail); bursty
    timestamps over 7.6 years; 1% of static pairs are planted triangles with a common burst."""
    rng = np.random.default_rng(seed)
    span = int(7.6 * YEAR)

    def mult_fn(r, k):
        heavy = r.random(k) >= 0.9749
        out = np.ones(k, dtype=np.int64)
        nh = int(heavy.sum())
        out[heavy] = np.minimum(r.zipf(1.8, nh), 10**5)
        return out

    src, dst, t, msd = _bursty_chung_lu(rng, n, 2.0, ms, mult_fn, span)
    return TemporalGraph(n, src, dst, t, name=f"plain_full_n{n}_ms{ms}",
                         meta={"deltas": [(d, d, d) for d in (600, 3600, 86400)]})


def delta_triple_like_batch(rng):
    """delta13 log-uniform over [60, 10^6]; delta12, delta23 uniform over {ceil(d13/4)..d13}."""
    d13 = int(round(np.exp(rng.uniform(np.log(60.0), np.log(1e6)))))
    lo = -(-d13 // 4)
    d12 = int(rng.integers(lo, d13 + 1))
    d23 = int(rng.integers(lo, d13 + 1))
    return d13, d12, d23


def batch_graph(index: int, seed: int = SEED_BASE + 3):
    """Graph `index` of the batched workload: n log-uniform over [10^3, 2*10^5], 10*n temporal
    edges, gamma=2.1, multiplicity min(Zipf(2), 10^4) with pairs added until 10*n edges,
    t ~ U{0..10^7-1}, orientation kept with probability 0.75."""
    rng = np.random.default_rng([seed, index])
    n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e5)))))
    m = 10 * n
    ms_draw = max(int(m / 5.0), 16)
    co = _cl_cdf(rng, n, 2.1, 2.0 * ms_draw)
    ci = _cl_cdf(rng, n, 2.1, 2.0 * ms_draw)
    u, v = _distinct_pairs(rng, n, co, ci, ms_draw)
    mult = np.minimum(rng.zipf(2.0, u.shape[0]), 10**4).astype(np.int64)
    cs = np.cumsum(mult)
    cut = min(int(np.searchsorted(cs, m, side="left")) + 1, u.shape[0])
    u, v, mult = u[:cut], v[:cut], mult[:cut]
    excess = int(mult.sum()) - m
    if excess > 0:
        mult[-1] -= excess
    _, src, dst = _expand(rng, u, v, mult, 0.75)
    t = rng.integers(0, 10**7, src.shape[0]).astype(np.int64)
    src, dst, t = _time_sorted(rng, src, dst, t)
    return TemporalGraph(n, src, dst, t, name=f"batch[{index}]_n{n}")


def batch_delta(index: int, seed: int = SEED_BASE + 3):
    """The delta triple of graph `index` of the batched workload."""
    return delta_triple_like_batch(np.random.default_rng([seed, index, 7]))


def served_stream(spans, duration_s: float = 60.0, rate: float = 2000.0,
                  seed: int = SEED_BASE + 4):
    """An open-loop Poisson query stream over resident graphs with time spans `spans`
    (list of (t_min, t_max)).  Each query picks a graph uniformly, a delta triple drawn as in the
    batched workload, and a window [t_a, t_b] with t_a uniform over the span and a width
    log-uniform over [1 day, span].  Returns a list of dicts sorted by arrival time (s)."""
    rng = np.random.default_rng(seed)
    k = int(rng.poisson(rate * duration_s))
    arr = np.sort(rng.random(k) * duration_s)
    out = []
    for i in range(k):
        g = int(rng.integers(0, len(spans)))
        tmin, tmax = spans[g]
        sp = max(int(tmax - tmin), 1)
        d13, d12, d23 = delta_triple_like_batch(rng)
        ta = int(tmin + rng.integers(0, sp + 1))
        lo_w = np.log(86400.0)
        hi_w = max(np.log(float(sp)), lo_w)
        width = int(round(np.exp(rng.uniform(lo_w, hi_w))))
        out.append({"arrival": float(arr[i]), "graph": g, "d13": d13, "d12": d12, "d23": d23,
                    "t_lo": ta, "t_hi": ta + width})
    return out


def clique_graph(k: int, seed: int, multi_frac: float = 0.02, max_mult: int = 5, t_range: int = 10**5,
                 noise_n: int = 0, noise_m: int = 0, all_mult: int = 0):
    """A k-clique (degeneracy k - 1) of temporal edges, for the dense extremes of the paper's
    inputs (large degeneracy, many triangles per static pair).  Each clique pair carries one
    temporal edge, or 2..max_mult of them with probability multi_frac (all_mult > 0: exactly
    all_mult on every pair); directions uniform; t ~ U{0..t_range-1}.  Optionally noise_m edges
    on noise_n further nodes, each joined to a random clique node or to another noise node."""
    rng = np.random.default_rng([SEED_BASE + 5, seed, k])
    iu, ju = np.triu_indices(k, 1)
    if all_mult:
        mult = np.full(iu.shape[0], all_mult, dtype=np.int64)
    else:
        mult = np.ones(iu.shape[0], dtype=np.int64)
        heavy = rng.random(iu.shape[0]) < multi_frac
        mult[heavy] = rng.integers(2, max_mult + 1, int(heavy.sum()))
    u = np.repeat(iu, mult).astype(np.int64)
    v = np.repeat(ju, mult).astype(np.int64)
    if noise_m:
        a = k + rng.integers(0, noise_n, noise_m)
        b = np.where(rng.random(noise_m) < 0.5, rng.integers(0, k, noise_m), k + rng.integers(0, noise_n, noise_m))
        ok = a != b
        u = np.concatenate([u, a[ok]])
        v = np.concatenate([v, b[ok]])
    flip = rng.random(u.shape[0]) < 0.5
    src = np.where(flip, v, u).astype(np.uint32)
    dst = np.where(flip, u, v).astype(np.uint32)
    t = rng.integers(0, t_range, src.shape[0]).astype(np.int64)
    perm = rng.permutation(src.shape[0])
    return TemporalGraph(k + noise_n, src[perm], dst[perm], t[perm], name=f"clique{k}(seed={seed})")


def contested_graph(seed: int, n_tri: int = 60, n: int = 400, span: int = 10**6, noise_m: int = 3000):
    """Triangles whose pairs carry many temporal edges in bursts, so that the number of edge pairs
    within d13 of each other grows from almost none to all of them across the deltas of a sweep:
    the shape where the medium path and the prefix procedures trade places.  Each of n_tri random
    triangles gets, per pair, a multiplicity from {1, 2, 7, 40, 150, 600} and its edges in the
    triangle's 1-4 sessions (uniform starts over the span shared by its three pairs, Exp(30) gaps);
    plus noise_m single edges between random nodes.  Directions uniform; the input is sorted by
    time with random tie order."""
    rng = np.random.default_rng([SEED_BASE + 6, seed])
    mults = np.array([1, 2, 7, 40, 150, 600])
    src, dst, ts = [], [], []
    for _ in range(n_tri):
        a, b, c = rng.choice(n, 3, replace=False)
        sess = int(rng.integers(1, 5))
        starts = rng.integers(0, span, sess)
        for (x, y) in ((a, b), (a, c), (b, c)):
            k = int(rng.choice(mults))
            which = rng.integers(0, sess, k)
            t = starts[which] + np.floor(rng.exponential(30.0, k)).astype(np.int64)
            flip = rng.random(k) < 0.5
            src.append(np.where(flip, y, x))
            dst.append(np.where(flip, x, y))
            ts.append(np.minimum(t, span))
    a = rng.integers(0, n, noise_m)
    b = rng.integers(0, n, noise_m)
    ok = a != b
    src.append(a[ok])
    dst.append(b[ok])
    ts.append(rng.integers(0, span, int(ok.sum())))
    src = np.concatenate(src).astype(np.uint32)
    dst = np.concatenate(dst).astype(np.uint32)
    t = np.concatenate(ts).astype(np.int64)
    src, dst, t = _time_sorted(rng, src, dst, t)
    return TemporalGraph(n, src, dst, t, name=f"contested(seed={seed})")


def long_lists_graph(seed: int, sizes=(5000, 3000, 700), t_range: int = 40000):
    """One triangle {0, 1, 2} whose pairs carry sizes[0], sizes[1], sizes[2] temporal edges (many
    prefix chunks per list, many equal timestamps), plus a pendant triangle {2, 3, 4} with 1, 2
    and 3 edges; t uniform over {0..t_range-1}, directions uniform."""
    rng = np.random.default_rng([SEED_BASE + 7, seed])
    pairs = [(0, 1), (0, 2), (1, 2), (2, 3), (3, 4), (2, 4)]
    ks = list(sizes) + [1, 2, 3]
    src, dst = [], []
    for (x, y), k in zip(pairs, ks):
        flip = rng.random(k) < 0.5
        src.append(np.where(flip, y, x))
        dst.append(np.where(flip, x, y))
    src = np.concatenate(src).astype(np.uint32)
    dst = np.concatenate(dst).astype(np.uint32)
    t = rng.integers(0, t_range, src.shape[0]).astype(np.int64)
    perm = rng.permutation(src.shape[0])
    return TemporalGraph(5, src[perm], dst[perm], t[perm], name=f"long_lists(seed={seed})")


def replicated(g: TemporalGraph, r: int) -> TemporalGraph:
    """Every temporal edge of g repeated r times, the copies adjacent in input order and sharing
    their timestamp.  The copies' keys (t, input index) keep the original edges' order, so every
    temporal triangle of g becomes exactly r^3 triangles here, for any deltas and window."""
    return TemporalGraph(g.n, np.repeat(g.src, r), np.repeat(g.dst, r), np.repeat(g.t, r),
                         name=f"{g.name}x{r}")


def disjoint_union(a: TemporalGraph, b: TemporalGraph) -> TemporalGraph:
    """a's edges then b's, b's nodes renumbered after a's (their triangles stay apart)."""
    return TemporalGraph(a.n + b.n, np.concatenate([a.src, b.src + np.uint32(a.n)]),
                         np.concatenate([a.dst, b.dst + np.uint32(a.n)]), np.concatenate([a.t, b.t]),
                         name=f"{a.name}+{b.name}")
