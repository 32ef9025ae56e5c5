"""GPU parity: counts through the C ABI against the CPU oracle, bit-exact (integer results).

Covers the light path, the heavy (prefix-count) path and mixes of both (the split is forced with
light_pair_cap), equal timestamps, self-loops, windows (empty, partial, whole), delta rewriting
(deltas out of order and past the span), the build products (core numbers, degeneracy bound on
out-degrees, triangle set, statistics) and determinism.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import INF, Built, say

pytestmark = pytest.mark.gpu

import paper_2106_02762_amd as dt  # noqa: E402

CAPS = [0, 1, 2, 3]   # split by the default caps, all light, all heavy, all medium


@pytest.fixture(scope="module")
def ctx():
    c = dt.dt_ctx_create(0)
    yield c
    dt.dt_ctx_destroy(c)


def _deltas(rng, tr, k=6):
    out = [(INF, INF, INF), (0, 0, 0), (tr, tr // 3, tr // 2), (tr // 4, tr, tr)]
    for _ in range(k):
        out.append(tuple(int(x) for x in rng.integers(0, tr + 3, 3)))
    return out


@pytest.mark.parametrize("cap", CAPS)
def test_tiny_multigraphs_match_oracle(ctx, cap):
    for seed in range(30):
        rng = np.random.default_rng(seed)
        g = synth.tiny_multigraph(seed, n=int(rng.integers(3, 9)), m=int(rng.integers(3, 40)),
                                  t_range=int(rng.integers(1, 12)))
        b = Built(ctx, g, g.name, cap)
        tr = int(g.t.max()) + 1
        for d in _deltas(rng, tr):
            lo, hi = (dt.INT64_MIN, INF) if rng.random() < 0.5 else \
                tuple(sorted(int(x) for x in rng.integers(-1, tr + 1, 2)))
            want = oracle.count(g.n, g.src, g.dst, g.t, *d, lo, hi)
            got = b.count(*d, lo, hi)
            assert (got == want).all(), (seed, cap, d, lo, hi, got, want)
        b.free()


@pytest.mark.parametrize("cap", CAPS)
def test_seed_graph_matches_oracle(ctx, cap):
    g = synth.seed_graph()
    b = Built(ctx, g, "seed50x300", cap)
    for d in [(300, 200, 150), (INF, INF, INF), (50, 50, 50), (0, 0, 0), (1000, 10, 990),
              (500, 900, 20)]:
        want = oracle.count(g.n, g.src, g.dst, g.t, *d)
        assert (b.count(*d) == want).all(), d
    for lo, hi in [(0, 999), (500, 1500), (1999, 1999), (-10, -1), (3000, 4000)]:
        want = oracle.count(g.n, g.src, g.dst, g.t, 300, 200, 150, lo, hi)
        assert (b.count(300, 200, 150, lo, hi) == want).all(), (lo, hi)
    b.free()


@pytest.mark.parametrize("cap", CAPS)
def test_plain_tiny_workload_delta_sweep(ctx, cap):
    g = synth.plain_tiny()
    b = Built(ctx, g, "plain_tiny", cap)
    for d in [(3600, 3600, 3600), (0, 0, 0), (10**4, 10**4, 10**4), (10**5, 10**5, 10**5),
              (INF, INF, INF), (10**5, 2 * 10**4, 7 * 10**4), (3 * 10**4, 10**5, 10**4)]:
        want = oracle.count(g.n, g.src, g.dst, g.t, *d)
        got = b.count(*d)
        assert (got == want).all(), (d, got, want)
    st = dt.dt_graph_stats(b.h)
    assert int(b.count(INF, INF, INF).sum()) == st["sum_sigma3"]
    b.free()


def test_heavy_multiplicities_with_ties(ctx):
    """Few pairs with hundreds of edges each and many equal timestamps: lists long enough that
    the heavy path spans several chunks and the searches have ragged tails."""
    rng = np.random.default_rng(7)
    n = 6
    pairs = [(0, 1), (0, 2), (1, 2), (2, 3), (1, 3), (0, 3), (3, 4), (4, 5), (3, 5)]
    sizes = [700, 300, 900, 5, 1, 260, 513, 2, 64]
    src, dst = [], []
    for (a, b), s in zip(pairs, sizes):
        flip = rng.random(s) < 0.4
        src += list(np.where(flip, b, a))
        dst += list(np.where(flip, a, b))
    src = np.array(src, dtype=np.uint32)
    dst = np.array(dst, dtype=np.uint32)
    t = rng.integers(0, 3000, src.shape[0]).astype(np.int64)
    perm = rng.permutation(src.shape[0])
    g = synth.TemporalGraph(n, src[perm], dst[perm], t[perm], name="heavy_ties")
    for cap in CAPS:
        b = Built(ctx, g, "heavy_ties", cap)
        for d in [(40, 30, 20), (300, 100, 250), (5, 5, 5), (INF, INF, INF), (0, 0, 0)]:
            want = oracle.count(n, g.src, g.dst, g.t, *d)
            assert (b.count(*d) == want).all(), (cap, d)
        want = oracle.count(n, g.src, g.dst, g.t, 100, 60, 70, 700, 2100)
        assert (b.count(100, 60, 70, 700, 2100) == want).all()
        b.free()


def test_build_products_match_oracle(ctx):
    for g in [synth.plain_tiny(), synth.seed_graph(), synth.tiny_multigraph(3, n=9, m=60, t_range=5)]:
        b = Built(ctx, g, g.name)
        ost, ocore = oracle.stats(g.n, g.src, g.dst, g.t, core=True)
        st = dt.dt_graph_stats(b.h)
        for k in ("m_static", "n_triangles", "degeneracy", "max_multiplicity", "self_loops",
                  "t_min", "t_max", "sum_sigma3"):
            gk = {"n_triangles": "n_static_triangles", "self_loops": "self_loops_dropped"}.get(k, k)
            if ost["m_window"] == 0 and k in ("t_min", "t_max"):
                continue
            assert st[gk] == ost[k], (g.name, k, st[gk], ost[k])
        core, rank = dt.dt_graph_order(b.h, g.n)
        assert (core == ocore).all()
        assert sorted(rank.tolist()) == list(range(g.n))
        assert st["max_out_degree"] <= st["degeneracy"]
        tri = dt.dt_graph_triangles(b.h)
        tri = tri[np.lexsort(tri.T[::-1])]
        otri = oracle.triangles(g.n, g.src, g.dst, g.t)
        assert tri.shape == otri.shape and (tri == otri).all()
        b.free()


def test_cells_sum_to_types_by_table2(ctx):
    from paper_tables import table2_psi
    psi = table2_psi()
    g = synth.seed_graph()
    for cap in CAPS:
        b = Built(ctx, g, "seed50x300", cap)
        for d in [(300, 200, 150), (INF, INF, INF)]:
            cells = dt.dt_count_cells(b.h, *d)
            types = b.count(*d)
            by = np.zeros(8, dtype=np.int64)
            for pi in range(1, 7):
                for rho in range(1, 9):
                    by[psi[pi][rho] - 1] += cells[pi - 1, rho - 1]
            assert (by == types).all()
        b.free()


def test_window_equals_filter_and_determinism(ctx):
    g = synth.plain_tiny()
    b = Built(ctx, g, "plain_tiny")
    for lo, hi in [(0, 10**6), (250_000, 600_000), (999_999, 999_999), (-5, 3), (400_000, 400_100)]:
        keep = (g.t >= lo) & (g.t <= hi)
        want = oracle.count(g.n, g.src[keep], g.dst[keep], g.t[keep], 10**5, 5 * 10**4, 8 * 10**4)
        got = b.count(10**5, 5 * 10**4, 8 * 10**4, lo, hi)
        assert (got == want).all(), (lo, hi)
    ref = b.count(10**5, 10**5, 10**5)
    for _ in range(10):
        assert (b.count(10**5, 10**5, 10**5) == ref).all()
    b.free()


def test_errors_are_reported(ctx):
    src = np.array([0, 1], np.uint32)
    dst = np.array([1, 5], np.uint32)
    t = np.array([1, 2], np.int64)
    say("error: node id >= n")
    with pytest.raises(dt.DtError) as e:
        dt.dt_graph_load(ctx, 3, src, dst, t)
    assert e.value.code == dt.DT_EINVAL
    g = dt.dt_graph_load(ctx, 6, src, dst, t)
    with pytest.raises(dt.DtError) as e:
        dt.dt_count(g, 1, 1, 1)
    assert e.value.code == dt.DT_ENOTBUILT
    dt.dt_graph_build(g)
    with pytest.raises(dt.DtError) as e:
        dt.dt_count(g, -1, 1, 1)
    assert e.value.code == dt.DT_EINVAL
    with pytest.raises(dt.DtError) as e:
        dt.dt_count(g, 1, 1, 1, 5, 4)
    assert e.value.code == dt.DT_EINVAL
    assert (dt.dt_count(g, 1, 1, 1) == 0).all()   # context still usable after errors
    dt.dt_graph_free(g)


def test_empty_and_degenerate_graphs(ctx):
    e = np.zeros(0, np.uint32)
    g = dt.dt_graph_load(ctx, 4, e, e, np.zeros(0, np.int64))
    dt.dt_graph_build(g)
    assert (dt.dt_count(g, INF, INF, INF) == 0).all()
    dt.dt_graph_free(g)
    loops = np.array([1, 2, 2], np.uint32)
    g = dt.dt_graph_load(ctx, 3, loops, loops, np.array([5, 6, 7], np.int64))
    dt.dt_graph_build(g)
    st = dt.dt_graph_stats(g)
    assert st["self_loops_dropped"] == 3 and st["m_static"] == 0
    assert (dt.dt_count(g, INF, INF, INF) == 0).all()
    dt.dt_graph_free(g)
    # one triangle, all timestamps equal: ties resolved by input order only
    src = np.array([0, 1, 2], np.uint32)
    dst = np.array([1, 2, 0], np.uint32)
    t = np.array([7, 7, 7], np.int64)
    b = Built(ctx, synth.TemporalGraph(3, src, dst, t, name="tie3"), "tie3")
    assert (b.count(0, 0, 0) == oracle.count(3, src, dst, t, 0, 0, 0)).all()
    b.free()
