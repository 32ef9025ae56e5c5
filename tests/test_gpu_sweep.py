"""GPU parity of delta sweeps (dt_count_sweep): k delta triples over one window counted in passes
of up to eight per visit of the triangle data must equal k separate counts, and the oracle's, on
every counting path (the default split, all light, all medium, all heavy), with and without a
window, for one pass, several passes and a single query; queries with different windows are
refused."""
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


SWEEP = [(0, 0, 0), (600, 600, 600), (3600, 3600, 3600), (7200, 1800, 5400), (86400, 86400, 86400),
         (30 * 86400, 20 * 86400, 20 * 86400), (86400, 10**7, 10**7), (INF, INF, INF),
         (3600, 3600, 0), (10**6, 4 * 10**5, 9 * 10**5), (1, 1, 1)]


def _check(b, deltas, lo=dt.INT64_MIN, hi=INF):
    say("sweep", b.name, len(deltas), "triples, window", lo, hi)
    got = dt.dt_count_sweep(b.h, deltas, lo, hi)
    assert got.shape == (len(deltas), 8)
    for j, d in enumerate(deltas):
        want = b.count(*d, lo, hi)
        assert (got[j] == want).all(), (b.name, d, lo, hi, got[j], want)
    return got


@pytest.mark.parametrize("path", [0, 1, 3])
def test_sweep_equals_single_counts(ctx, path):
    g = synth.plain_full(n=60_000, ms=800_000)
    b = Built(ctx, g, "scaled plain_full", path=path)
    t0, t1 = int(g.t.min()), int(g.t.max())
    got = _check(b, SWEEP)                       # two passes (8 + 3)
    _check(b, SWEEP[:8])                         # one full pass
    _check(b, SWEEP[2:3])                        # a single query
    _check(b, SWEEP, t0 + (t1 - t0) // 3, t0 + (t1 - t0) // 2)
    if path == 0:   # the oracle for two triples of the sweep
        for j in (2, 5):
            want = oracle.count(g.n, g.src, g.dst, g.t, *SWEEP[j])
            assert (got[j] == want).all(), (SWEEP[j], got[j], want)
    b.free()


def test_sweep_heavy_path_and_ties(ctx):
    for seed in range(3):
        g = synth.tiny_multigraph(seed, n=12, m=400, t_range=50)
        for path in (0, 2):
            b = Built(ctx, g, f"tiny multigraph {seed}", path=path)
            deltas = [(d13, d12, d23) for d13 in (0, 3, 10, 40) for d12, d23 in ((d13, d13), (d13 // 2, d13))]
            got = _check(b, deltas)
            for j in (0, 3, 7):
                want = oracle.count(g.n, g.src, g.dst, g.t, *deltas[j])
                assert (got[j] == want).all(), (seed, path, deltas[j])
            _check(b, deltas[:5], 10, 30)
            b.free()


def test_sweep_rejects_mixed_windows(ctx):
    g = synth.seed_graph()
    b = Built(ctx, g, "seed graph")
    qs = [(100, 100, 100, 0, 1000), (100, 100, 100, 0, 999)]
    arr = (dt.dt_query * 2)(*[dt.make_query(*q) for q in qs])
    out = np.zeros((2, 8), dtype=np.int64)
    rc = dt.library().dt_count_sweep(b.h, 2, arr, out.ctypes.data)
    assert rc == dt.DT_EINVAL
    b.free()
