"""dt_count_noalloc (no allocation; scratch in the library's fixed per-device array) against
dt_count_async on the same graphs and queries, bit-exact: two calls in a row, the second on a
smaller graph, through the heavy (prefix-count) path whose prefix arrays live in that scratch
and through the default split; a count whose scratch need exceeds the array is refused."""
import numpy as np
import pytest

import synth
from gpu_common import INF, Built, say

pytestmark = pytest.mark.gpu

import paper_2106_02762_amd as dt  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = dt.dt_ctx_create(0)
    yield c
    dt.dt_ctx_destroy(c)


def _pair(b, q, torch):
    """(dt_count_async result, dt_count_noalloc result) for query q on graph b."""
    dev = torch.device("cuda:0")
    ref = torch.full((8,), -7, dtype=torch.int64, device=dev)
    got = torch.full((8,), -7, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    dt.dt_count_async(b.h, q, ref.data_ptr())
    dt.dt_count_noalloc(b.h, q, got.data_ptr())
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_equals_async_two_calls(ctx):
    import torch
    big = Built(ctx, synth.plain_tiny(), "plain_tiny heavy", 2)         # every triangle on the heavy path
    small = Built(ctx, synth.seed_graph(), "seed50x300 heavy", 2)
    default = Built(ctx, synth.plain_tiny(), "plain_tiny default")
    for b, q in [(big, dt.make_query(10**5, 5 * 10**4, 8 * 10**4)),
                 (small, dt.make_query(300, 200, 150)),
                 (default, dt.make_query(10**5, 10**5, 10**5, 250_000, 600_000)),
                 (small, dt.make_query(INF, INF, INF))]:
        say("noalloc vs async", b.name)
        ref, got = _pair(b, q, torch)
        assert (ref >= 0).all() and (got == ref).all(), (b.name, ref, got)
    for b in (big, small, default):
        b.free()


def test_noalloc_refuses_oversized_scratch(ctx):
    import torch
    g = synth.clique_graph(100, 2, all_mult=3)   # 161,700 heavy triangles: ~100 MB of prefix arrays
    b = Built(ctx, g, g.name, 2)
    out = torch.full((8,), -7, dtype=torch.int64, device=torch.device("cuda:0"))
    torch.cuda.synchronize()
    with pytest.raises(dt.DtError) as e:
        dt.dt_count_noalloc(b.h, dt.make_query(3600, 3600, 3600), out.data_ptr())
    assert e.value.code == dt.DT_ENOMEM
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == -7).all()
    # the library stays usable, and a count that fits works right after
    small = Built(ctx, synth.seed_graph(), "seed50x300")
    ref, got = _pair(small, dt.make_query(300, 200, 150), torch)
    assert (got == ref).all()
    small.free()
    b.free()
