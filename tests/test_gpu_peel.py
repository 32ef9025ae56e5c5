"""GPU parity of the degeneracy ordering of Section 3, by both methods.  The second one (h-index core
numbers, then every shell peeled at once) on the graph of shapes and one power-law graph; the
default level-by-level peel in its regimes:
the whole peel on the cooperative grid (peel_tail = 1), the whole peel in one workgroup (graphs of
at most 16320 vertices), the grid handing its last vertices to one workgroup, and (on a 600K-vertex
graph) the full-width grid for the first levels before the narrow one.  A graph of shapes covers
the second method's row kinds and histogram passes (hubs of 2,000 and 20,000 neighbours, a clique,
a long path whose bounds and removals travel one hop per phase, isolated vertices).  Core numbers
must equal the oracle's exactly (they are unique, unlike the ordering), the ordering must be a
permutation, and every vertex must have at most core(v) neighbours after it in the ordering (the
out-degree bound Theorem 1 uses)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import INF, say

pytestmark = pytest.mark.gpu

import paper_2106_02762_amd as dt  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = dt.dt_ctx_create(0)
    yield c
    dt.dt_ctx_destroy(c)


def _static_pairs(g):
    a = np.minimum(g.src, g.dst).astype(np.int64)
    b = np.maximum(g.src, g.dst).astype(np.int64)
    keep = a != b
    key = np.unique(a[keep] * g.n + b[keep])
    return key // g.n, key % g.n


def _check(ctx, g, method, peel_tail, ocore, pairs, query):
    say("ordering", g.name, "method", method, "peel_tail", peel_tail)
    h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
    try:
        dt.dt_graph_set_tuning(h, peel_tail=peel_tail, order_method=method)
        dt.dt_graph_build(h)
        st = dt.dt_graph_stats(h)
        core, rank = dt.dt_graph_order(h, g.n)
        assert (core == ocore).all(), (g.name, method, peel_tail, int((core != ocore).sum()))
        assert st["degeneracy"] == int(ocore.max())
        assert np.array_equal(np.sort(rank), np.arange(g.n, dtype=rank.dtype))
        u, v = pairs
        first = np.where(rank[u] < rank[v], u, v)   # each pair points away from this endpoint
        outdeg = np.bincount(first, minlength=g.n)
        assert (outdeg <= core).all(), (g.name, method, peel_tail)
        assert st["max_out_degree"] == int(outdeg.max())
        return dt.dt_count(h, *query)
    finally:
        dt.dt_graph_free(h)


class _G:
    def __init__(self, name, n, src, dst, t):
        self.name, self.n, self.src, self.dst, self.t = name, n, src, dst, t


def shapes_graph(seed=7):
    """Hubs of 20,000 and 2,000 leaves (leaves paired into triangles with their hub), a 60-clique
    joined to the second hub, a 3,000-vertex path, 100 isolated vertices; 1-3 temporal edges per
    pair at random times."""
    rng = np.random.default_rng(seed)
    pairs = []
    nxt = 0

    def new(k):
        nonlocal nxt
        ids = np.arange(nxt, nxt + k)
        nxt += k
        return ids

    for leaves in (20_000, 2_000):
        hub = new(1)[0]
        lv = new(leaves)
        pairs += [(hub, x) for x in lv]
        pairs += [(lv[i], lv[i + 1]) for i in range(0, leaves - 1, 2)]
    hub2 = nxt - 2_001
    cl = new(60)
    pairs += [(int(a), int(b)) for i, a in enumerate(cl) for b in cl[i + 1:]]
    pairs += [(hub2, int(a)) for a in cl]
    path = new(3_000)
    pairs += [(int(path[i]), int(path[i + 1])) for i in range(len(path) - 1)]
    new(100)
    src, dst = [], []
    for a, b in pairs:
        for _ in range(int(rng.integers(1, 4))):
            if rng.random() < 0.5:
                a, b = b, a
            src.append(a)
            dst.append(b)
    src = np.array(src, np.uint32)
    dst = np.array(dst, np.uint32)
    perm = rng.permutation(nxt).astype(np.uint32)   # ids not in construction order
    t = rng.integers(0, 100_000, size=src.shape[0]).astype(np.int64)
    return _G("shapes", nxt, perm[src], perm[dst], t)


@pytest.mark.parametrize("name", ["large", "scaled", "batch5", "plain_tiny", "tiny", "shapes"])
def test_peel_regimes_match_oracle(ctx, name):
    if name == "shapes":
        g = shapes_graph()
        tails = [0, 1]
        q = (3600, 3600, 3600, dt.INT64_MIN, INF)
    elif name == "large":
        g = synth.plain_full(n=600_000, ms=8_000_000)    # the whole grid first, then 32 blocks
        tails = [0, 1]
        q = (3600, 3600, 3600, dt.INT64_MIN, INF)
    elif name == "scaled":
        g = synth.plain_full(n=60_000, ms=800_000)       # grid, then one workgroup
        tails = [0, 1, 100, 16320]
        q = (3600, 3600, 3600, dt.INT64_MIN, INF)
    elif name == "batch5":
        g = synth.batch_graph(5)                          # n = 48,229
        tails = [0, 1, 5000]
        q = (3600, 1800, 3600, dt.INT64_MIN, INF)
    elif name == "plain_tiny":
        g = synth.plain_tiny()                            # n = 1,000: one workgroup throughout
        tails = [0, 1, 10]
        q = (10**5, 5 * 10**4, 8 * 10**4, dt.INT64_MIN, INF)
    else:
        g = synth.tiny_multigraph(3, n=9, m=60, t_range=5)
        tails = [0, 1, 2]
        q = (3, 2, 2, dt.INT64_MIN, INF)
    _, ocore = oracle.stats(g.n, g.src, g.dst, g.t, core=True)
    pairs = _static_pairs(g)
    want = oracle.count(g.n, g.src, g.dst, g.t, *q)
    # the second method (h-index core numbers, slower than the level peel on every graph measured)
    # on the graph of shapes that covers its row kinds and on one power-law graph only
    methods = [(1, 0)] if name in ("shapes", "scaled") else []
    for method, pt in methods + [(0, pt) for pt in tails]:
        got = _check(ctx, g, method, pt, ocore, pairs, q)
        assert (got == want).all(), (name, method, pt, got, want)


def test_peel_tail_is_validated(ctx):
    g = synth.seed_graph()
    h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
    try:
        with pytest.raises(dt.DtError) as e:
            dt.dt_graph_set_tuning(h, peel_tail=16321)
        assert e.value.code == dt.DT_EINVAL
        with pytest.raises(dt.DtError) as e:
            dt.dt_graph_set_tuning(h, order_method=2)
        assert e.value.code == dt.DT_EINVAL
    finally:
        dt.dt_graph_free(h)
