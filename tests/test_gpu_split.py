"""The medium / prefix-procedure split by d13, the chunked prefix pass and the work bound.

- Contested triangles (bursty multi-edge pairs) change path with d13: counts equal the oracle at
  every delta of a sweep across the levels, whole span and windowed, under three cost weights and
  the forced paths, and in sweeps and batches.
- Long lists (5,000 / 3,000 / 700 edges, many equal timestamps): the prefix pass spans many chunks
  per list and carries between them; windows cut lists inside chunks.
- A short and a long source pair: the medium path's entries split the long one into chunks.
- Theorem 1's work bound (Section 5): the instrumented count's visits stay within
  2 * 48 * degeneracy * m' at every d13 up to infinity, with counts equal to dt_count's.
- The autotuner: a graph of 2^20 static triangles or more is tuned on its first build and a
  second graph of its size class reuses the choice; counts stay exact.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import INF, Built, say

pytestmark = pytest.mark.gpu

import paper_2106_02762_amd as dt  # noqa: E402

SWEEP = [0, 1, 10, 60, 100, 1000, 3600, 10**5, 10**6, INF]


@pytest.fixture(scope="module")
def ctx():
    c = dt.dt_ctx_create(0)
    yield c
    dt.dt_ctx_destroy(c)


@pytest.mark.parametrize("pct", [0, 25, 400])
def test_contested_triangles_across_levels(ctx, pct):
    g = synth.contested_graph(1)
    b = Built(ctx, g, g.name)
    if pct:
        dt.dt_graph_set_tuning(b.h, medium_cost_pct=pct)
    st = dt.dt_graph_stats(b.h)
    say("contested", st["n_contested_triangles"], "medium", st["n_medium_triangles"], "heavy", st["n_heavy_triangles"])
    assert st["n_contested_triangles"] > 0
    for d in SWEEP:
        want = oracle.count(g.n, g.src, g.dst, g.t, d, d, d)
        assert (b.count(d, d, d) == want).all(), (pct, d)
    for d in [(10**5, 100, 1000), (300, 10**5, 50), (5000, 2000, 4000)]:
        want = oracle.count(g.n, g.src, g.dst, g.t, *d)
        assert (b.count(*d) == want).all(), (pct, d)
    for lo, hi in [(0, 300_000), (250_000, 250_500), (600_000, 10**6)]:
        for d in (10, 3600, INF):
            want = oracle.count(g.n, g.src, g.dst, g.t, d, d, d, lo, hi)
            assert (b.count(d, d, d, lo, hi) == want).all(), (pct, d, lo, hi)
    # a sweep across the levels, whole span and windowed, equals the separate counts
    deltas = [(d, d, d) for d in (1, 60, 1000, 10**5, INF)]
    for lo, hi in [(dt.INT64_MIN, INF), (100_000, 900_000)]:
        got = dt.dt_count_sweep(b.h, deltas, lo, hi)
        for j, d in enumerate(deltas):
            assert (got[j] == b.count(*d, lo, hi)).all(), (pct, d, lo, hi)
    # batched: one query per level band, windows mixed in
    qs = [dt.make_query(d, d, d) for d in SWEEP] + [dt.make_query(3600, 3600, 3600, 250_000, 750_000)]
    got = dt.dt_count_batch(ctx, [b.h] * len(qs), qs)
    for i, q in enumerate(qs):
        assert (got[i] == dt.dt_count(b.h, q.d13, q.d12, q.d23, q.t_lo, q.t_hi)).all(), i
    b.free()


@pytest.mark.parametrize("path", [0, 2, 3])
def test_long_lists_prefix_chunks(ctx, path):
    g = synth.long_lists_graph(1)
    b = Built(ctx, g, g.name, path)
    for d in [(3000, 1000, 2500), (40, 30, 20), (0, 0, 0), (10**4, 10**4, 10**4)]:
        want = oracle.count(g.n, g.src, g.dst, g.t, *d)
        assert (b.count(*d) == want).all(), (path, d)
    for lo, hi in [(1000, 1000), (12345, 23456), (0, 300), (39000, 50000)]:
        want = oracle.count(g.n, g.src, g.dst, g.t, 3000, 1000, 2500, lo, hi)
        assert (b.count(3000, 1000, 2500, lo, hi) == want).all(), (path, lo, hi)
    if path != 3:
        # infinite deltas: the product identity (the oracle would enumerate 10^10 triples)
        st = dt.dt_graph_stats(b.h)
        assert int(b.count(INF, INF, INF).sum()) == st["sum_sigma3"]
    b.free()


@pytest.mark.parametrize("path", [0, 3])
@pytest.mark.parametrize("sizes", [(3, 700, 900), (1, 2000, 40), (2, 513, 1025)])
def test_medium_inner_chunks(ctx, path, sizes):
    """Triangles with a short and a long source pair: the medium path's entries cover chunks of 512
    inner edges (a chunk may straddle the inner pair's two direction runs, and a list of 513 or
    1025 edges ends in a one-edge chunk).  Counts equal the oracle's across d13, with windows, in a
    sweep and in a batch."""
    g = synth.long_lists_graph(3, sizes=sizes, t_range=5000)
    b = Built(ctx, g, g.name, path)
    for d in [0, 1, 30, 300, 2000, INF]:
        want = oracle.count(g.n, g.src, g.dst, g.t, d, d, d)
        assert (b.count(d, d, d) == want).all(), (path, sizes, d)
    for d in [(4000, 100, 3900), (500, 400, 60)]:
        for lo, hi in [(dt.INT64_MIN, INF), (700, 3100), (2500, 2600)]:
            want = oracle.count(g.n, g.src, g.dst, g.t, *d, lo, hi)
            assert (b.count(*d, lo, hi) == want).all(), (path, sizes, d, lo, hi)
    deltas = [(d, d, d) for d in (5, 300, INF)]
    got = dt.dt_count_sweep(b.h, deltas)
    for j, d in enumerate(deltas):
        assert (got[j] == b.count(*d)).all(), (path, sizes, d)
    qs = [dt.make_query(d, d, d) for d in (5, 300, INF)] + [dt.make_query(300, 300, 300, 700, 3100)]
    got = dt.dt_count_batch(ctx, [b.h] * len(qs), qs)
    for i, q in enumerate(qs):
        assert (got[i] == dt.dt_count(b.h, q.d13, q.d12, q.d23, q.t_lo, q.t_hi)).all(), (path, sizes, i)
    b.free()


def test_visits_within_the_work_bound(ctx):
    cases = [synth.contested_graph(2), synth.long_lists_graph(2), synth.plain_tiny(),
             synth.clique_graph(100, 2, all_mult=3), synth.plain_medium()]
    for g in cases:
        b = Built(ctx, g, g.name)
        st = dt.dt_graph_stats(b.h)
        kappa = st["degeneracy"]
        for d in [600, 3600, 86400, 10**6, INF]:
            for lo, hi in [(dt.INT64_MIN, INF), (int(g.t.min()), int(g.t.min()) + (int(g.t.max()) - int(g.t.min())) // 3)]:
                got, visits = dt.dt_count_visits(b.h, d, d, d, lo, hi)
                assert (got == b.count(d, d, d, lo, hi)).all(), (g.name, d)
                m_win = int(((g.t >= lo) & (g.t <= hi) & (g.src != g.dst)).sum())
                say("visits", g.name, d, lo, hi, visits, "bound", 2 * 48 * kappa * m_win)
                assert visits <= 2 * 48 * kappa * m_win, (g.name, d, visits, kappa, m_win)
        b.free()


def test_autotuner_tunes_once_per_size_class(ctx):
    g1 = synth.clique_graph(190, 3, noise_n=200, noise_m=1500, multi_frac=0.05)
    g2 = synth.clique_graph(190, 4, noise_n=200, noise_m=1500, multi_frac=0.05)
    b1 = Built(ctx, g1, g1.name)
    st1 = dt.dt_graph_stats(b1.h)
    assert st1["n_static_triangles"] >= 1 << 20
    assert st1["autotuned"] == 1
    assert st1["light_pair_cap_used"] in (2, 4, 8) and st1["medium_cost_pct_used"] in (25, 100, 400)
    b2 = Built(ctx, g2, g2.name)
    st2 = dt.dt_graph_stats(b2.h)
    assert st2["autotuned"] == 1
    for k in ("light_pair_cap_used", "medium_cost_pct_used", "light_blocks_per_cu", "medium_blocks_per_cu"):
        assert st2[k] == st1[k], k
    for b, g in ((b1, g1), (b2, g2)):
        for d in [(3600, 3600, 3600), (20000, 5000, 18000)]:
            want = oracle.count(g.n, g.src, g.dst, g.t, *d)
            assert (b.count(*d) == want).all(), (g.name, d)
    # never tuning: the defaults
    dt.dt_graph_set_tuning(b2.h, autotune=1)
    dt.dt_graph_build(b2.h)
    st3 = dt.dt_graph_stats(b2.h)
    assert st3["autotuned"] == 0 and st3["light_pair_cap_used"] == 4 and st3["medium_cost_pct_used"] == 100
    b1.free()
    b2.free()
