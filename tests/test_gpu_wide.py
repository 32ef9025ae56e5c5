"""Counts of graphs whose sum of multiplicity products reaches 2^63 (128-bit accumulation).

Repeating every temporal edge r times (copies adjacent in input order, equal timestamps) multiplies
every count by exactly r^3: each temporal triangle of the original becomes r^3 triangles, and the
copies' keys keep the original edges' order.  A K4 with 1,400 edges per pair repeated 1,000 times
has a sum of multiplicity products of about 1.1e19 >= 2^63 while each type count at infinite
deltas stays below 2^63; joined with a contested graph on separate nodes (unit, light, medium and
prefix-procedure triangles), every path runs with 128-bit partials.  Repeated 3,000 times, the
type counts at infinite deltas reach 2^63 and are refused, while short deltas still fit.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import INF, Built, say

pytestmark = pytest.mark.gpu

import paper_2106_02762_amd as dt  # noqa: E402

R = 1000
DELTAS = [(0, 0, 0), (60, 60, 60), (3600, 3600, 3600), (86400, 86400, 86400), (5000, 2000, 4000),
          (10**6, 10**6, 10**6), (INF, INF, INF)]
WINDOWS = [(dt.INT64_MIN, INF), (200_000, 700_000)]


_MEMO = {}


def _k4():
    return synth.clique_graph(4, 7, all_mult=1400, t_range=10**6)


def _oracle(g, d, lo, hi):
    # the K4's counts at long deltas take the oracle seconds: each is computed once
    k = (g.name, d, lo, hi)
    if k not in _MEMO:
        _MEMO[k] = [int(x) for x in oracle.count(g.n, g.src, g.dst, g.t, *d, lo, hi)]
    return _MEMO[k]


def _expected(small, rest, r, d, lo, hi):
    want = [x * r ** 3 for x in _oracle(small, d, lo, hi)]
    if rest is not None:
        want = [w + x for w, x in zip(want, _oracle(rest, d, lo, hi))]
    return want


@pytest.fixture(scope="module")
def ctx():
    c = dt.dt_ctx_create(0)
    yield c
    dt.dt_ctx_destroy(c)


def test_wide_counts_equal_the_scaled_oracle(ctx):
    small, noise = _k4(), synth.contested_graph(3)
    g = synth.disjoint_union(synth.replicated(small, R), noise)
    b = Built(ctx, g, g.name)
    st = dt.dt_graph_stats(b.h)
    say("sum_sigma3", st["sum_sigma3"], "unit", st["n_unit_triangles"], "light", st["n_light_triangles"],
        "medium", st["n_medium_triangles"], "heavy", st["n_heavy_triangles"])
    assert st["sum_sigma3"] >= 1 << 63
    assert min(st["n_unit_triangles"], st["n_light_triangles"], st["n_medium_triangles"],
               st["n_heavy_triangles"]) > 0
    for lo, hi in WINDOWS:
        for d in DELTAS:
            want = _expected(small, noise, R, d, lo, hi)
            assert [int(x) for x in b.count(*d, lo, hi)] == want, (d, lo, hi)
    # whole span at infinite deltas: every triple, so the types sum to the sum of products
    assert sum(int(x) for x in b.count(INF, INF, INF)) == st["sum_sigma3"]
    for d in [(3600, 3600, 3600), (INF, INF, INF)]:
        got, visits = dt.dt_count_visits(b.h, *d)
        assert [int(x) for x in got] == _expected(small, noise, R, d, dt.INT64_MIN, INF), d
        assert visits > 0
    for path in (2, 3):
        dt.dt_graph_set_tuning(b.h, force_path=path)
        for d in [(60, 60, 60), (86400, 86400, 86400), (INF, INF, INF)]:
            assert [int(x) for x in b.count(*d)] == _expected(small, noise, R, d, dt.INT64_MIN, INF), (path, d)
    dt.dt_graph_set_tuning(b.h, force_path=0)
    # the calls that return int64 sums without a 128-bit pass refuse such a graph
    import torch
    q = dt.make_query(3600, 3600, 3600)
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    for name, call in [("cells", lambda: dt.dt_count_cells(b.h, 3600, 3600, 3600)),
                       ("sweep", lambda: dt.dt_count_sweep(b.h, [(3600, 3600, 3600)])),
                       ("batch", lambda: dt.dt_count_batch(ctx, [b.h], [q])),
                       ("async", lambda: dt.dt_count_async(b.h, q, out.data_ptr())),
                       ("noalloc", lambda: dt.dt_count_noalloc(b.h, q, out.data_ptr()))]:
        say("refused", name)
        with pytest.raises(dt.DtError) as e:
            call()
        assert e.value.code == dt.DT_EOVERFLOW, name
    # the one-pass count (its rest goes through a 128-bit pass)
    for d in [(3600, 3600, 3600), (INF, INF, INF)]:
        say("oneshot", d)
        got = dt.dt_count_oneshot(b.h, *d)
        assert [int(x) for x in got] == _expected(small, noise, R, d, dt.INT64_MIN, INF), d
    b.free()


def test_type_counts_beyond_int64_are_refused(ctx):
    small = _k4()
    r = 3000
    g = synth.replicated(small, r)
    b = Built(ctx, g, g.name)
    want_inf = _expected(small, None, r, (INF, INF, INF), dt.INT64_MIN, INF)
    assert max(want_inf) >= 1 << 63
    say("count inf (refused)")
    with pytest.raises(dt.DtError) as e:
        dt.dt_count(b.h, INF, INF, INF)
    assert e.value.code == dt.DT_EOVERFLOW
    for d in [(600, 600, 600), (3600, 3600, 3600)]:
        want = _expected(small, None, r, d, dt.INT64_MIN, INF)
        assert max(want) < 1 << 63
        assert [int(x) for x in b.count(*d)] == want, d
    b.free()
