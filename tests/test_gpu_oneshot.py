"""GPU parity of the one-shot count (dt_count_oneshot): ordering, orientation and an enumeration
pass that counts unit and light triangles as it finds them, the rest handed to the medium and heavy
paths.  Its result must equal the oracle's and the cached path's (dt_graph_build + dt_count) for
every split of the triangles (light caps, medium caps that send the rest to the heavy path), with
and without windows; it drops any earlier build."""
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


def _oneshot(h, name, *q):
    say("oneshot", name, *q)
    return dt.dt_count_oneshot(h, *q)


def test_scaled_graph_matches_oracle_and_cached_path(ctx):
    g = synth.plain_full(n=60_000, ms=800_000)
    t0, t1 = int(g.t.min()), int(g.t.max())
    h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
    try:
        cases = [(3600, 3600, 3600, dt.INT64_MIN, INF), (30 * 86400, 20 * 86400, 20 * 86400, dt.INT64_MIN, INF),
                 (86400, 86400, 86400, t0 + (t1 - t0) // 4, t0 + (t1 - t0) // 2), (0, 0, 0, dt.INT64_MIN, INF)]
        for q in cases:
            got = _oneshot(h, "scaled", *q)
            want = oracle.count(g.n, g.src, g.dst, g.t, *q)
            assert (got == want).all(), (q, got, want)
        with pytest.raises(dt.DtError) as e:
            dt.dt_count(h, 3600, 3600, 3600)
        assert e.value.code == dt.DT_ENOTBUILT
        say("build after oneshot")
        dt.dt_graph_build(h)
        for q in cases:
            assert (dt.dt_count(h, *q) == oracle.count(g.n, g.src, g.dst, g.t, *q)).all(), q
        got = _oneshot(h, "scaled after build", *cases[0])   # replaces the build
        assert (got == oracle.count(g.n, g.src, g.dst, g.t, *cases[0])).all()
    finally:
        dt.dt_graph_free(h)


@pytest.mark.parametrize("caps", [(0, 0), (1, 0), (64, 0), (4, 1)])
def test_multigraphs_every_split(ctx, caps):
    light_cap, medium_cap = caps
    for seed in range(4):
        g = synth.tiny_multigraph(seed, n=12, m=400, t_range=50)
        h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
        try:
            dt.dt_graph_set_tuning(h, light_pair_cap=light_cap, medium_pair_cap=medium_cap)
            for q in [(0, 0, 0, dt.INT64_MIN, INF), (10, 5, 10, dt.INT64_MIN, INF), (40, 40, 40, 10, 30),
                      (7, 7, 1, dt.INT64_MIN, INF), (10**9, 10**9, 10**9, dt.INT64_MIN, INF)]:
                got = _oneshot(h, f"multigraph {seed} caps {caps}", *q)
                want = oracle.count(g.n, g.src, g.dst, g.t, *q)
                assert (got == want).all(), (seed, caps, q, got, want)
        finally:
            dt.dt_graph_free(h)


def test_second_ordering_method(ctx):
    """With the h-index ordering (order_method 1) the one-shot count, and a build and count after
    it, still equal the oracle's (counts do not depend on the degeneracy ordering chosen)."""
    g = synth.plain_full(n=60_000, ms=800_000)
    h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
    try:
        dt.dt_graph_set_tuning(h, order_method=1)
        q = (3600, 1800, 3600, dt.INT64_MIN, INF)
        want = oracle.count(g.n, g.src, g.dst, g.t, *q)
        assert (_oneshot(h, "scaled, h-index ordering", *q) == want).all()
        say("build with the h-index ordering")
        dt.dt_graph_build(h)
        assert (dt.dt_count(h, *q) == want).all()
    finally:
        dt.dt_graph_free(h)


def test_batch_graph_and_degenerate_inputs(ctx):
    g = synth.batch_graph(3)
    h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
    try:
        for q in [(10**6, 6 * 10**5, 8 * 10**5, dt.INT64_MIN, INF), (10**6, 10**6, 10**6, 2 * 10**6, 5 * 10**6)]:
            got = _oneshot(h, "batch_graph 3", *q)
            assert (got == oracle.count(g.n, g.src, g.dst, g.t, *q)).all(), q
        # a window outside the span: zeros, nothing run
        assert (_oneshot(h, "empty window", 100, 100, 100, -10, -5) == 0).all()
    finally:
        dt.dt_graph_free(h)
    # a graph without triangles, and one without edges
    src = np.array([0, 1, 2], np.uint32)
    dst = np.array([1, 2, 3], np.uint32)
    t = np.array([1, 2, 3], np.int64)
    h = dt.dt_graph_load(ctx, 4, src, dst, t)
    try:
        assert (_oneshot(h, "path graph", 10, 10, 10) == 0).all()
    finally:
        dt.dt_graph_free(h)
    h = dt.dt_graph_load(ctx, 4, src[:0], dst[:0], t[:0])
    try:
        assert (_oneshot(h, "no edges", 10, 10, 10) == 0).all()
    finally:
        dt.dt_graph_free(h)
