"""GPU parity of windowed counts through the window index of the light and medium lists.

Those lists are ordered by a cell of two time slices (the latest first-edge time and the earliest
last-edge time over a triangle's three pairs), and a windowed query visits only the cells that can
hold a triangle inside its window.  The skipped cells must hold nothing the window can see, so
every windowed count equals the oracle's count on the filtered edge list, whichever path the
triangles take, for windows placed on and around slice boundaries, tiny and wide windows, and
through the batched launch as through the single-query one."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import Built, say

pytestmark = pytest.mark.gpu

import paper_2106_02762_amd as dt  # noqa: E402

SLICES = 32


@pytest.fixture(scope="module")
def ctx():
    c = dt.dt_ctx_create(0)
    yield c
    dt.dt_ctx_destroy(c)


def _windows(g, rng):
    t0, t1 = int(g.t.min()), int(g.t.max())
    span = t1 - t0
    s = 0
    while (span >> s) >= SLICES:
        s += 1
    w = []
    for k in sorted({1, 5, 17, span >> s}):   # on and around slice boundaries inside the span
        b = t0 + (k << s)
        w += [(b - 1, b), (b, b + (1 << s) - 1), (b - 3600, b + 3600), (t0, b - 1), (b, t1)]
    for _ in range(16):        # widths log-uniform over [1 day, span]
        lo = int(t0 + rng.integers(0, span + 1))
        width = int(np.exp(rng.uniform(np.log(86400.0), np.log(float(span)))))
        w.append((lo, lo + width))
    w += [(t0, t0), (t1, t1), (t0 - 10, t0 + 86400), (t1 - 86400, t1 + 10)]
    assert all(lo <= hi for lo, hi in w)
    return w


def _want(g, d, lo, hi):
    keep = (g.t >= lo) & (g.t <= hi)
    return oracle.count(g.n, g.src[keep], g.dst[keep], g.t[keep], *d)


@pytest.mark.parametrize("path", [0, 1, 3])
def test_windowed_counts_match_oracle(ctx, path):
    g = synth.plain_full(n=60_000, ms=800_000)
    rng = np.random.default_rng(11)
    b = Built(ctx, g, "scaled plain_full", path=path)
    st = dt.dt_graph_stats(b.h)
    if path == 0:
        assert st["n_light_triangles"] > 1000 and st["n_medium_triangles"] > 10
    d = (30 * 86400, 20 * 86400, 20 * 86400)
    wins = _windows(g, rng)
    for lo, hi in wins:
        got = b.count(*d, lo, hi)
        want = _want(g, d, lo, hi)
        assert (got == want).all(), (path, lo, hi, got, want)
    # the same windows in one batched launch
    say("batch of", len(wins), "windows, path", path)
    qs = [dt.make_query(*d, lo, hi) for lo, hi in wins]
    out = dt.dt_count_batch(ctx, [b.h] * len(wins), qs)
    for i, (lo, hi) in enumerate(wins):
        assert (out[i] == b.count(*d, lo, hi)).all(), (path, lo, hi)
    b.free()


def test_windowed_multigraph_with_ties(ctx):
    # heavy multiplicities and equal timestamps: light, medium and heavy triangles together
    g = synth.batch_graph(3)
    rng = np.random.default_rng(12)
    b = Built(ctx, g, "batch_graph 3")
    d = (10**6, 6 * 10**5, 8 * 10**5)
    for lo, hi in _windows(g, rng)[:24]:
        got = b.count(*d, lo, hi)
        want = _want(g, d, lo, hi)
        assert (got == want).all(), (lo, hi, got, want)
    b.free()
