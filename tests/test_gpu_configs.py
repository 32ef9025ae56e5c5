"""GPU parity on the workload shapes and on the branches the small graphs never reach.

- The medium plain workload (n = 10^6, 10^7 temporal edges, Zipf(2) multiplicity on every pair),
  whole span, at two symmetric delta triples and an asymmetric one, plus a window: bit-exact
  against the oracle (Definition 1, Section 1.1).
- A 520-clique with multi-edge noise: degeneracy 519, so the first vertices of the ordering have
  more out-neighbours than one wavefront's LDS slice holds (the global-memory enumeration
  branch), and 23M triangles on 155K pairs (the enumeration's rerun at the counted size).
- A 100-clique with three temporal edges on every pair: 161,700 triangles on 4,950 pairs, all of
  them past the light rule, through the cached build (every path) and the one-shot pass (whose
  list of medium triangles overflows its first size).
- Ranks past 2^26 (2^26 + 4096 vertices, the edges among the last ids): the orientation's runs of
  at most 64 entries then take the bitonic network instead of 32-bit key counting; a 90-clique
  gives runs longer than 64 as well.
- dt_count_async on the context's stream and on a foreign stream, into device and pinned memory.
- Sixteen graphs of the 512-graph batched workload in one dt_count_batch call, each with its own
  delta triple, against the oracle.
- The full-size workload, whose triangle list is written in reserved stretches with empty
  entries between them: triangle count, statistics and whole-span counts against the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import INF, Built, say

pytestmark = pytest.mark.gpu

import paper_2106_02762_amd as dt  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = dt.dt_ctx_create(0)
    yield c
    dt.dt_ctx_destroy(c)


def _sorted_tris(a):
    return a[np.lexsort(a.T[::-1])]


def test_medium_workload_whole_span_matches_oracle(ctx):
    g = synth.plain_medium()
    b = Built(ctx, g, g.name)
    st = dt.dt_graph_stats(b.h)
    ost = oracle.stats(g.n, g.src, g.dst, g.t)
    for k in ("m_static", "degeneracy", "max_multiplicity", "sum_sigma3"):
        assert st[k] == ost[k], (k, st[k], ost[k])
    assert st["n_static_triangles"] == ost["n_triangles"]
    lo = int(g.t.min())
    for d in [(3600, 3600, 3600), (86400, 86400, 86400), (86400, 3600, 43200)]:
        want = oracle.count(g.n, g.src, g.dst, g.t, *d)
        got = b.count(*d)
        say("medium", d, got.tolist(), want.tolist())
        assert (got == want).all(), (d, got, want)
    # a window over the second year
    wlo, whi = lo + synth.graphs.YEAR, lo + 2 * synth.graphs.YEAR
    want = oracle.count(g.n, g.src, g.dst, g.t, 86400, 86400, 86400, wlo, whi)
    assert (b.count(86400, 86400, 86400, wlo, whi) == want).all()
    b.free()


def test_degeneracy_above_the_lds_slice(ctx):
    g = synth.clique_graph(520, 1, noise_n=3000, noise_m=20000)
    b = Built(ctx, g, g.name)
    st = dt.dt_graph_stats(b.h)
    ost = oracle.stats(g.n, g.src, g.dst, g.t)
    assert st["degeneracy"] == ost["degeneracy"] == 519
    assert 512 < st["max_out_degree"] <= st["degeneracy"]
    assert st["n_static_triangles"] == ost["n_triangles"]
    assert st["n_static_triangles"] > 4 * st["m_static"]   # the enumeration ran again at its size
    say("triangle set", st["n_static_triangles"])
    tri = _sorted_tris(dt.dt_graph_triangles(b.h))
    otri = oracle.triangles(g.n, g.src, g.dst, g.t)
    assert tri.shape == otri.shape and (tri == otri).all()
    del tri, otri
    for d in [(3600, 3600, 3600), (20000, 5000, 18000), (INF, INF, INF)]:
        want = oracle.count(g.n, g.src, g.dst, g.t, *d)
        assert (b.count(*d) == want).all(), d
    assert int(b.count(INF, INF, INF).sum()) == st["sum_sigma3"]
    say("one-shot", g.name)
    want = oracle.count(g.n, g.src, g.dst, g.t, 20000, 5000, 18000)
    assert (dt.dt_count_oneshot(b.h, 20000, 5000, 18000) == want).all()
    b.free()


@pytest.mark.parametrize("path", [0, 1, 2, 3])
def test_dense_clique_more_triangles_than_pairs(ctx, path):
    g = synth.clique_graph(100, 2, all_mult=3)
    b = Built(ctx, g, g.name, path)
    st = dt.dt_graph_stats(b.h)
    assert st["n_static_triangles"] == 161700 > max(4 * st["m_static"], 65536)
    for d in [(3600, 3600, 3600), (20000, 5000, 18000), (0, 0, 0), (INF, INF, INF)]:
        want = oracle.count(g.n, g.src, g.dst, g.t, *d)
        assert (b.count(*d) == want).all(), (path, d)
    if path == 0:
        # one-shot: every triangle has sigma_uv sigma_uw = 9 > the light rule, so all 161,700 go
        # to its rest list (first sized for 65,536) and the fused pass runs again
        for d in [(3600, 3600, 3600), (20000, 5000, 18000)]:
            want = oracle.count(g.n, g.src, g.dst, g.t, *d)
            say("one-shot", g.name, d)
            assert (dt.dt_count_oneshot(b.h, *d) == want).all(), d
        dt.dt_graph_build(b.h)
        want = oracle.count(g.n, g.src, g.dst, g.t, 20000, 5000, 18000)
        assert (b.count(20000, 5000, 18000) == want).all()
    b.free()


def test_ranks_beyond_2_26(ctx):
    n = (1 << 26) + 4096
    rng = np.random.default_rng(5)
    ids = n - 1 - rng.permutation(4096)[:200]
    src, dst = [], []
    for k, off in ((90, 0), (40, 90)):
        c = ids[off:off + k]
        a, b = np.triu_indices(k, 1)
        src.append(c[a])
        dst.append(c[b])
    x, y = rng.choice(ids, 600), rng.choice(ids, 600)
    src.append(x[x != y])
    dst.append(y[x != y])
    src, dst = np.concatenate(src).astype(np.uint32), np.concatenate(dst).astype(np.uint32)
    flip = rng.random(src.shape[0]) < 0.5
    src, dst = np.where(flip, dst, src), np.where(flip, src, dst)
    t = rng.integers(0, 10000, src.shape[0]).astype(np.int64)
    o = np.argsort(t, kind="stable")
    g = synth.TemporalGraph(n, src[o], dst[o], t[o], name="ranks_past_2^26")
    b = Built(ctx, g, g.name)
    st = dt.dt_graph_stats(b.h)
    assert st["max_out_degree"] > 64
    for d in [(3000, 2000, 2500), (INF, INF, INF), (40, 30, 20)]:
        want = oracle.count(g.n, g.src, g.dst, g.t, *d)
        assert (b.count(*d) == want).all(), d
    say("one-shot", g.name)
    want = oracle.count(g.n, g.src, g.dst, g.t, 3000, 2000, 2500)
    assert (dt.dt_count_oneshot(b.h, 3000, 2000, 2500) == want).all()
    b.free()


def test_count_async_streams_and_memory(ctx):
    import torch
    g = synth.plain_tiny()
    b = Built(ctx, g, g.name)
    deltas = [(10**5, 5 * 10**4, 8 * 10**4), (3600, 3600, 3600), (INF, INF, INF), (10**4, 10**4, 10**4)]
    want = [b.count(*d) for d in deltas]
    dev = torch.device("cuda:0")
    # the context's stream (NULL), device outputs; a synchronous count after them orders the stream
    outs = [torch.full((8,), -1, dtype=torch.int64, device=dev) for _ in deltas]
    torch.cuda.synchronize()   # the fills run on torch's stream, which the library's does not follow
    for d, o in zip(deltas, outs):
        say("async ctx stream", d)
        dt.dt_count_async(b.h, dt.make_query(*d), o.data_ptr())
    dt.dt_count(b.h, 1, 1, 1)
    for o, w in zip(outs, want):
        assert (o.cpu().numpy() == w).all()
    # a foreign stream, pinned host outputs, with a windowed query among them
    s = torch.cuda.Stream(device=dev)
    pins = [torch.full((8,), -1, dtype=torch.int64).pin_memory() for _ in range(len(deltas) + 1)]
    for d, p in zip(deltas, pins):
        say("async foreign stream", d)
        dt.dt_count_async(b.h, dt.make_query(*d), p.data_ptr(), s.cuda_stream)
    dt.dt_count_async(b.h, dt.make_query(10**5, 10**5, 10**5, 250_000, 600_000), pins[-1].data_ptr(), s.cuda_stream)
    s.synchronize()
    for p, w in zip(pins, want):
        assert (p.numpy() == w).all()
    keep = (g.t >= 250_000) & (g.t <= 600_000)
    assert (pins[-1].numpy() == oracle.count(g.n, g.src[keep], g.dst[keep], g.t[keep], 10**5, 10**5, 10**5)).all()
    # a foreign-stream count followed at once by one on the context's stream (shared scratch)
    o2 = torch.full((8,), -1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    dt.dt_count_async(b.h, dt.make_query(*deltas[0]), o2.data_ptr(), s.cuda_stream)
    assert (b.count(*deltas[1]) == want[1]).all()
    s.synchronize()
    assert (o2.cpu().numpy() == want[0]).all()
    b.free()


def test_batched_workload_graphs_match_oracle(ctx):
    idx = list(range(0, 512, 32))
    gs = [synth.batch_graph(i) for i in idx]
    ds = [synth.batch_delta(i) for i in idx]
    hs = []
    for g in gs:
        say("build", g.name, g.m)
        h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
        dt.dt_graph_build(h)
        hs.append(h)
    say("batch of", len(hs))
    got = dt.dt_count_batch(ctx, hs, [dt.make_query(*d) for d in ds])
    for i, (g, d) in enumerate(zip(gs, ds)):
        want = oracle.count(g.n, g.src, g.dst, g.t, *d)
        assert (got[i] == want).all(), (g.name, d, got[i], want)
    for h in hs:
        dt.dt_graph_free(h)


def test_full_workload_list_written_in_stretches(ctx):
    """The full-size workload (61M edges, 67M static triangles) is large enough that the
    enumeration's wavefronts reserve list positions in stretches and leave empty entries: the
    triangle count, the sum of multiplicity products and the degeneracy equal the oracle's, and the
    whole-span counts at (3600, 3600, 3600) equal the oracle's (Definition 1)."""
    g = synth.plain_full()
    b = Built(ctx, g, g.name)
    st = dt.dt_graph_stats(b.h)
    say("oracle stats", g.name)
    ost = oracle.stats(g.n, g.src, g.dst, g.t)
    assert st["n_static_triangles"] == ost["n_triangles"]
    assert st["sum_sigma3"] == ost["sum_sigma3"]
    assert st["degeneracy"] == ost["degeneracy"]
    say("oracle count", g.name)
    want = oracle.count(g.n, g.src, g.dst, g.t, 3600, 3600, 3600)
    assert (b.count(3600, 3600, 3600) == want).all()
    b.free()
