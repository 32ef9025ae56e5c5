"""Device memory of a context: the HBM budget is enforced (DT_ENOMEM, never an overrun), rebuilds
reuse the context's cached blocks instead of growing, and results do not depend on whether a
buffer came fresh from the device or from the cache."""
import pytest

import oracle
import synth
from gpu_common import say

pytestmark = pytest.mark.gpu

import paper_2106_02762_amd as dt  # noqa: E402


def test_budget_and_block_reuse():
    budget = 48 << 20
    ctx = dt.dt_ctx_create(0, hbm_budget_bytes=budget)
    try:
        g = synth.plain_tiny()
        say("budgeted build", g.name)
        h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
        dt.dt_graph_build(h)
        want = oracle.count(g.n, g.src, g.dst, g.t, 10**5, 5 * 10**4, 8 * 10**4)
        assert (dt.dt_count(h, 10**5, 5 * 10**4, 8 * 10**4) == want).all()
        used1, b = dt.dt_ctx_memory(ctx)
        assert b == budget and used1 <= budget
        held = []
        for _ in range(6):
            dt.dt_graph_build(h)   # the same sizes again: served from the cache
            assert (dt.dt_count(h, 10**5, 5 * 10**4, 8 * 10**4) == want).all()
            held.append(dt.dt_ctx_memory(ctx)[0])
        # best fit may take a larger cached block once, but the holdings settle instead of growing
        assert max(held) <= 1.5 * used1 and held[-1] <= held[2], (used1, held)

        big = synth.plain_full(n=60_000, ms=800_000)   # needs far more than the budget
        say("over-budget load", big.name)
        with pytest.raises(dt.DtError) as e:
            hb = dt.dt_graph_load(ctx, big.n, big.src, big.dst, big.t)
            try:
                dt.dt_graph_build(hb)
            finally:
                dt.dt_graph_free(hb)
        assert e.value.code == dt.DT_ENOMEM
        used3, _ = dt.dt_ctx_memory(ctx)
        assert used3 <= budget
        # the resident graph is untouched
        assert (dt.dt_count(h, 10**5, 5 * 10**4, 8 * 10**4) == want).all()
        dt.dt_graph_free(h)
    finally:
        dt.dt_ctx_destroy(ctx)
