"""Serving more graphs than the HBM budget holds: with host swapping, a server whose budget fits
two of four graphs answers queries on all four, moving the least recently used idle graphs to host
memory and back; every result equals the same query counted alone before admission, and the bytes
in HBM never pass the budget.  After the server stops, graphs left in host memory count again."""
import numpy as np
import pytest

import synth
from gpu_common import INF, say

pytestmark = pytest.mark.gpu

import paper_2106_02762_amd as dt  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = dt.dt_ctx_create(0)
    yield c
    dt.dt_ctx_destroy(c)


def _queries(g, k, rng):
    tmin, tmax = int(g.t.min()), int(g.t.max())
    span = max(tmax - tmin, 1)
    out = []
    for _ in range(k):
        d = [int(rng.integers(0, span + 2)) for _ in range(3)]
        if rng.random() < 0.2:
            d = [INF] * 3
        if rng.random() < 0.5:
            lo, hi = dt.INT64_MIN, INF
        else:
            a = tmin + int(rng.integers(0, span + 1))
            lo, hi = a, a + int(rng.integers(0, span + 1))
        out.append((*d, lo, hi))
    return out


def test_swapping_server_answers_beyond_its_budget(ctx):
    gs = [synth.plain_tiny(synth.SEED_BASE + 40 + i) for i in range(4)]
    hs = []
    for g in gs:
        say("build", g.name, g.m)
        h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
        dt.dt_graph_build(h)
        hs.append(h)
    rng = np.random.default_rng(5)
    qs = [_queries(g, 12, rng) for g in gs]
    want = [[dt.dt_count(h, *q) for q in qq] for h, qq in zip(hs, qs)]

    # the graphs' device bytes, from a server without a budget
    srv = dt.dt_server_start(ctx)
    sizes = [dt.dt_server_graph_info(srv, dt.dt_server_add_graph(srv, h))[1] for h in hs]
    dt.dt_server_stop(srv)
    s = sorted(sizes)
    budget = s[-1] + s[-2] + 4096
    say("sizes", sizes, "budget", budget)
    assert s[0] + s[1] + s[2] > budget   # no three fit

    # without swapping the third graph is refused
    srv = dt.dt_server_start(ctx, hbm_budget_bytes=budget)
    dt.dt_server_add_graph(srv, hs[0])
    dt.dt_server_add_graph(srv, hs[1])
    with pytest.raises(dt.DtError) as e:
        for h in hs[2:]:
            dt.dt_server_add_graph(srv, h)
    assert e.value.code == dt.DT_ENOMEM
    dt.dt_server_stop(srv)

    srv = dt.dt_server_start(ctx, hbm_budget_bytes=budget, max_batch=8, swap_to_host=1)
    ids = [dt.dt_server_add_graph(srv, h) for h in hs]
    st = dt.dt_server_stats(srv)
    say("admitted", st)
    assert st["graphs"] == 4 and st["resident_graphs"] <= 2 and st["resident_bytes"] <= budget
    assert not all(dt.dt_server_graph_info(srv, i)[0] for i in ids)
    # while held, direct calls that touch the device are refused; statistics still answer
    with pytest.raises(dt.DtError) as e:
        dt.dt_count(hs[0], 3600, 3600, 3600)
    assert e.value.code == dt.DT_EBUSY
    assert dt.dt_graph_stats(hs[3])["m"] == gs[3].m
    with pytest.raises(dt.DtError) as e:
        dt.dt_server_add_graph(srv, hs[0])
    assert e.value.code == dt.DT_EBUSY

    # one graph at a time, cycling through all four: each turn swaps
    for r in range(3):
        for gi in (0, 2, 1, 3):
            q = qs[gi][r]
            got = dt.dt_server_wait(srv, dt.dt_server_submit(srv, ids[gi], *q))
            assert (got == want[gi][r]).all(), (gi, r)
            st = dt.dt_server_stats(srv)
            assert st["resident_bytes"] <= budget and st["resident_graphs"] <= 2, st
    # bursts mixing all four graphs (batches take what fits; the rest waits for room)
    for burst in range(2):
        order = [(gi, r) for gi in range(4) for r in range(3 + 4 * burst, 7 + 4 * burst)]
        rng.shuffle(order)
        tickets = [(gi, r, dt.dt_server_submit(srv, ids[gi], *qs[gi][r])) for gi, r in order]
        for gi, r, t in tickets:
            got = dt.dt_server_wait(srv, t)
            assert (got == want[gi][r]).all(), (burst, gi, r)
        st = dt.dt_server_stats(srv)
        assert st["resident_bytes"] <= budget, st
    st = dt.dt_server_stats(srv)
    say("after", st)
    assert st["swap_ins"] >= 6 and st["swap_outs"] >= 6
    assert st["queries_done"] == 12 + 32
    dt.dt_server_stop(srv)

    # back with the caller: graphs left in host memory return on their next use
    for h, qq, ww in zip(hs, qs, want):
        for q, w in zip(qq[:3], ww[:3]):
            assert (dt.dt_count(h, *q) == w).all()
    for h in hs:
        dt.dt_graph_free(h)
