"""Batched and served counting: every query's result in a batch or in the served mix equals the
same query counted alone (exact integers), and the serving loop's admission, deadlines, timeouts
and error isolation behave as documented."""
import threading

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


def _heavy_graph():
    rng = np.random.default_rng(11)
    pairs = [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3), (0, 3)]
    sizes = [600, 700, 400, 3, 90, 1]
    src, dst = [], []
    for (a, b), s in zip(pairs, sizes):
        flip = rng.random(s) < 0.5
        src += list(np.where(flip, b, a))
        dst += list(np.where(flip, a, b))
    src = np.array(src, np.uint32)
    dst = np.array(dst, np.uint32)
    t = rng.integers(0, 5000, src.shape[0]).astype(np.int64)
    return synth.TemporalGraph(4, src, dst, t, name="heavy4")


@pytest.fixture(scope="module")
def graphs(ctx):
    gs = [synth.seed_graph(), synth.plain_tiny(), _heavy_graph()]
    gs += [synth.tiny_multigraph(s, n=8, m=50, t_range=20) for s in range(4)]
    gs += [synth.batch_graph(i) for i in (5, 17, 40)]
    gs.append(synth.TemporalGraph(5, np.zeros(0, np.uint32), np.zeros(0, np.uint32),
                                  np.zeros(0, np.int64), name="empty"))
    hs = []
    for i, g in enumerate(gs):
        say("build", g.name, g.m)
        h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
        dt.dt_graph_build(h)
        if i == 2:
            dt.dt_graph_set_tuning(h, force_path=2)   # every triangle on the prefix-count path
        if i == 3:
            dt.dt_graph_set_tuning(h, force_path=3)   # every triangle on the medium path
        hs.append(h)
    yield list(zip(gs, hs))
    for h in hs:
        dt.dt_graph_free(h)


def _queries(gs, k, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(k):
        gi = int(rng.integers(0, len(gs)))
        g = gs[gi][0]
        tmax = int(g.t.max()) if g.m else 10
        tmin = int(g.t.min()) if g.m else 0
        span = max(tmax - tmin, 1)
        d13 = int(rng.integers(0, span + 2))
        d12 = int(rng.integers(0, span + 2))
        d23 = int(rng.integers(0, span + 2))
        if rng.random() < 0.15:
            d13 = d12 = d23 = INF
        r = rng.random()
        if r < 0.5:
            lo, hi = dt.INT64_MIN, INF
        elif r < 0.9:
            a = tmin + int(rng.integers(0, span + 1))
            lo, hi = a, a + int(rng.integers(0, span + 1))
        else:
            lo, hi = tmax + 5, tmax + 10   # empty window
        out.append((gi, (d13, d12, d23, lo, hi)))
    return out


def test_batch_equals_alone(ctx, graphs):
    qs = _queries(graphs, 300, 1)
    alone = [dt.dt_count(graphs[gi][1], *q) for gi, q in qs]
    say("batch of", len(qs))
    got = dt.dt_count_batch(ctx, [graphs[gi][1] for gi, _ in qs], [dt.make_query(*q) for _, q in qs])
    for i, (gi, q) in enumerate(qs):
        assert (got[i] == alone[i]).all(), (i, graphs[gi][0].name, q, got[i], alone[i])
    # the same batch again (the tuned, captured launch is replayed) and a smaller one
    got2 = dt.dt_count_batch(ctx, [graphs[gi][1] for gi, _ in qs], [dt.make_query(*q) for _, q in qs])
    assert (got2 == got).all()
    small = qs[:7]
    got3 = dt.dt_count_batch(ctx, [graphs[gi][1] for gi, _ in small], [dt.make_query(*q) for _, q in small])
    assert (got3 == got[:7]).all()
    assert dt.dt_count_batch(ctx, [], []).shape == (0, 8)


def test_batch_spot_checks_against_oracle(ctx, graphs):
    qs = [(0, (300, 200, 150, dt.INT64_MIN, INF)), (2, (40, 30, 20, dt.INT64_MIN, INF)),
          (1, (10**5, 5 * 10**4, 8 * 10**4, 250_000, 600_000))]
    got = dt.dt_count_batch(ctx, [graphs[gi][1] for gi, _ in qs], [dt.make_query(*q) for _, q in qs])
    for i, (gi, q) in enumerate(qs):
        g = graphs[gi][0]
        assert (got[i] == oracle.count(g.n, g.src, g.dst, g.t, *q)).all()


def test_server_results_alone_equal_mix(ctx, graphs):
    qs = _queries(graphs, 400, 2)
    alone = [dt.dt_count(graphs[gi][1], *q) for gi, q in qs]
    srv = dt.dt_server_start(ctx, max_batch=64)
    ids = [dt.dt_server_add_graph(srv, h) for _, h in graphs]
    results = {}
    errors = []

    def client(part):
        try:
            tickets = [(i, dt.dt_server_submit(srv, ids[qs[i][0]], *qs[i][1])) for i in part]
            for i, t in tickets:
                results[i] = dt.dt_server_wait(srv, t)
        except Exception as e:   # noqa: BLE001
            errors.append(e)

    say("serving", len(qs), "queries from 4 threads")
    th = [threading.Thread(target=client, args=(list(range(j, len(qs), 4)),)) for j in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    dt.dt_server_stop(srv)
    assert not errors, errors
    for i in range(len(qs)):
        assert (results[i] == alone[i]).all(), (i, qs[i])


def test_server_admission_and_errors(ctx, graphs):
    srv = dt.dt_server_start(ctx, hbm_budget_bytes=4096)
    with pytest.raises(dt.DtError) as e:
        dt.dt_server_add_graph(srv, graphs[1][1])
    assert e.value.code == dt.DT_ENOMEM
    dt.dt_server_stop(srv)

    srv = dt.dt_server_start(ctx)
    gid = dt.dt_server_add_graph(srv, graphs[0][1])
    good = dt.dt_server_submit(srv, gid, 300, 200, 150)
    with pytest.raises(dt.DtError) as e:
        dt.dt_server_submit(srv, gid, -1, 5, 5)            # invalid query refused alone
    assert e.value.code == dt.DT_EINVAL
    with pytest.raises(dt.DtError) as e:
        dt.dt_server_submit(srv, 99, 1, 1, 1)              # unknown graph
    assert e.value.code == dt.DT_EINVAL
    t2 = dt.dt_server_submit(srv, gid, INF, INF, INF)
    try:
        r = dt.dt_server_wait(srv, t2, timeout_ns=0)       # done or still pending, never lost
    except dt.DtError as e:
        assert e.code == dt.DT_ETIMEDOUT
        r = dt.dt_server_wait(srv, t2)
    g = graphs[0][0]
    assert (r == oracle.count(g.n, g.src, g.dst, g.t, INF, INF, INF)).all()
    assert (dt.dt_server_wait(srv, good) == dt.dt_count(graphs[0][1], 300, 200, 150)).all()
    with pytest.raises(dt.DtError):
        dt.dt_server_wait(srv, good)                       # a ticket is collected once
    dt.dt_server_stop(srv)


def test_server_deadline_and_stop(ctx, graphs):
    srv = dt.dt_server_start(ctx, deadline_ns=1)
    gid = dt.dt_server_add_graph(srv, graphs[1][1])
    tickets = [dt.dt_server_submit(srv, gid, 3600, 3600, 3600) for _ in range(20)]
    codes = []
    for t in tickets:
        try:
            dt.dt_server_wait(srv, t)
            codes.append(0)
        except dt.DtError as e:
            codes.append(e.code)
    assert all(c in (0, dt.DT_ETIMEDOUT) for c in codes) and dt.DT_ETIMEDOUT in codes
    dt.dt_server_stop(srv)
    srv = dt.dt_server_start(ctx)
    gid = dt.dt_server_add_graph(srv, graphs[1][1])
    for _ in range(50):
        dt.dt_server_submit(srv, gid, 3600, 3600, 3600)
    dt.dt_server_stop(srv)   # drains what was submitted, then returns
