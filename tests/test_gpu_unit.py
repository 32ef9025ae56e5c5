"""GPU parity of the unit-triangle path: triangles with one temporal edge on each pair are stored
as records with their ordering and orientation fixed at build time and counted by testing the
three times against the query.  Checked against the oracle (exact integers) on a graph where most
of ~10^6 triangles are unit triangles, with windows narrow enough that the t1-ordered index skips
most records, through single counts, the cells diagnostic and batches; and on a graph whose time
span is too wide for the record format, where the path must stay off.  The same graph's triangle
list is checked against the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import INF, Built, say

pytestmark = pytest.mark.gpu

import paper_2106_02762_amd as dt  # noqa: E402

DAY = 86_400


@pytest.fixture(scope="module")
def ctx():
    c = dt.dt_ctx_create(0)
    yield c
    dt.dt_ctx_destroy(c)


@pytest.fixture(scope="module")
def scaled(ctx):
    # the full-size workload's recipe at n = 60,000 and 800,000 static pairs: ~1.2M temporal
    # edges, ~960K static triangles, mostly with one edge per pair
    g = synth.plain_full(n=60_000, ms=800_000)
    b = Built(ctx, g, g.name)
    yield g, b
    b.free()


def _windows(g, rng, k):
    t0, t1 = int(g.t.min()), int(g.t.max())
    out = [(dt.INT64_MIN, INF), (t0, t1), (t0 + 1, t1 - 1), (t1 + 1, t1 + 5), (t0 - 10, t0)]
    for _ in range(k):
        width = int(np.exp(rng.uniform(np.log(DAY), np.log(t1 - t0))))
        a = int(rng.integers(t0 - DAY, t1))
        out.append((a, a + width))
    return out


def test_unit_records_cover_most_triangles(scaled):
    g, b = scaled
    st = dt.dt_graph_stats(b.h)
    # a contested triangle is in both the medium and the heavy list (each query takes one of them)
    parts = st["n_unit_triangles"] + st["n_light_triangles"] + st["n_medium_triangles"] + \
        st["n_heavy_triangles"] - st["n_contested_triangles"]
    assert parts == st["n_static_triangles"]
    assert st["n_unit_triangles"] > 0.8 * st["n_static_triangles"], st
    assert st["alg_bytes_unit"] == 16 * st["n_unit_triangles"]


def test_triangle_list_matches_oracle(scaled):
    """The build's triangle list on this graph (about a million triangles, written by thousands of
    wavefronts in no particular order) holds exactly the oracle's triangles."""
    g, b = scaled
    st = dt.dt_graph_stats(b.h)
    tri = dt.dt_graph_triangles(b.h)
    assert tri.shape == (st["n_static_triangles"], 3)
    tri = tri[np.lexsort(tri.T[::-1])]
    otri = oracle.triangles(g.n, g.src, g.dst, g.t)
    assert tri.shape == otri.shape and (tri == otri).all()


def test_unit_windows_match_oracle(scaled):
    g, b = scaled
    rng = np.random.default_rng(7)
    deltas = [(3600, 3600, 3600), (INF, INF, INF), (DAY, 600, DAY), (0, 0, 0), (7 * DAY, DAY, 3 * DAY)]
    for lo, hi in _windows(g, rng, 24):
        d = deltas[int(rng.integers(0, len(deltas)))]
        want = oracle.count(g.n, g.src, g.dst, g.t, *d, lo, hi)
        got = b.count(*d, lo, hi)
        assert (got == want).all(), (d, lo, hi, got, want)


def test_unit_cells_equal_light_path_cells(scaled):
    # the same handle re-split (the ordering, and so the cell names, stay those of its build)
    g, b = scaled
    qs = [(3600, 3600, 3600, dt.INT64_MIN, INF),
          (DAY, DAY, DAY, int(g.t.min()) + 30 * DAY, int(g.t.min()) + 400 * DAY)]
    c_unit = []
    for q in qs:
        say("cells", q)
        c_unit.append((dt.dt_count_cells(b.h, *q), dt.dt_count(b.h, *q)))
    dt.dt_graph_set_tuning(b.h, force_path=1)
    try:
        assert dt.dt_graph_stats(b.h)["n_unit_triangles"] == 0
        for q, (cells, counts) in zip(qs, c_unit):
            say("cells, all light", q)
            assert (dt.dt_count_cells(b.h, *q) == cells).all(), q
            assert (dt.dt_count(b.h, *q) == counts).all(), q
    finally:
        dt.dt_graph_set_tuning(b.h, force_path=0)


def test_unit_batch_equals_alone(ctx, scaled):
    g, b = scaled
    rng = np.random.default_rng(8)
    qs = []
    for lo, hi in _windows(g, rng, 60):
        d = tuple(int(x) for x in rng.integers(0, 3 * DAY, 3))
        qs.append((*d, lo, hi))
    alone = [dt.dt_count(b.h, *q) for q in qs]
    say("unit batch of", len(qs))
    got = dt.dt_count_batch(ctx, [b.h] * len(qs), [dt.make_query(*q) for q in qs])
    for i, q in enumerate(qs):
        assert (got[i] == alone[i]).all(), (i, q, got[i], alone[i])


def test_tuning_round_trip_restores_unit_records(scaled):
    g, b = scaled
    q = (DAY, 3600, DAY, int(g.t.min()) + 100 * DAY, int(g.t.min()) + 200 * DAY)
    before = dt.dt_count(b.h, *q)
    n_unit = dt.dt_graph_stats(b.h)["n_unit_triangles"]
    say("force medium, then back")
    dt.dt_graph_set_tuning(b.h, force_path=3)
    assert dt.dt_graph_stats(b.h)["n_unit_triangles"] == 0
    assert (dt.dt_count(b.h, *q) == before).all()
    dt.dt_graph_set_tuning(b.h, force_path=0)
    assert dt.dt_graph_stats(b.h)["n_unit_triangles"] == n_unit
    assert (dt.dt_count(b.h, *q) == before).all()


def test_wide_span_keeps_unit_path_off(ctx):
    # times stretched 10^4-fold: the span (~10^10) exceeds 2^31, so no record format fits and
    # every triangle, unit ones included, is counted by the pairwise paths
    g0 = synth.plain_tiny()
    g = synth.TemporalGraph(g0.n, g0.src, g0.dst, g0.t * 10_000, name="plain-tiny-wide-span")
    b = Built(ctx, g, g.name)
    try:
        assert dt.dt_graph_stats(b.h)["n_unit_triangles"] == 0
        for d in [(10**9, 5 * 10**8, 8 * 10**8), (INF, INF, INF), (10**8, 10**8, 10**8)]:
            want = oracle.count(g.n, g.src, g.dst, g.t, *d)
            assert (b.count(*d) == want).all(), d
    finally:
        b.free()
