"""CPU DOTTT (oracle/cpu_dottt.c): the paper's own procedures -- degeneracy ordering, orientation,
triangle listing, the prefix-count procedures for {v,w} third, second and first, Table 2 -- run
sequentially.  It shares no code with the plain oracle, so agreement on graphs with many equal
timestamps, asymmetric and degenerate deltas and windows checks the readings of those procedures
(ties by input position, delta normalisation) against Definition 1 itself.  Also checked without
the oracle: the infinite-delta identity (every ordered triple of edges on a triangle's three pairs
is counted once) and invariance under relabelling the vertices."""
import numpy as np
import pytest

import oracle
import synth

DELTAS = [(0, 0, 0), (1, 1, 1), (3, 2, 2), (5, 1, 4), (2, 5, 1), (4, 4, 1), (10**9, 10**9, 10**9)]


@pytest.mark.parametrize("seed", range(40))
def test_tiny_multigraphs_with_ties(seed):
    g = synth.tiny_multigraph(seed, n=8, m=40, t_range=6)
    for d in DELTAS:
        want = oracle.count(g.n, g.src, g.dst, g.t, *d)
        got = oracle.cpu_dottt(g.n, g.src, g.dst, g.t, *d)
        assert (got == want).all(), (seed, d, got, want)


@pytest.mark.parametrize("seed", range(8))
def test_long_lists_and_windows(seed):
    g = synth.tiny_multigraph(seed, n=12, m=400, t_range=50)
    for d in [(0, 0, 0), (3, 2, 2), (10, 5, 10), (40, 40, 40), (40, 10, 35), (7, 7, 1)]:
        for w in [(oracle.INT64_MIN, oracle.INT64_MAX), (10, 30), (25, 25), (-5, 3)]:
            want = oracle.count(g.n, g.src, g.dst, g.t, *d, *w)
            got = oracle.cpu_dottt(g.n, g.src, g.dst, g.t, *d, *w)
            assert (got == want).all(), (seed, d, w, got, want)


def test_seed_graph_and_tiny_workload():
    g = synth.seed_graph()
    for d in [(0, 0, 0), (100, 50, 80), (500, 500, 500), (2000, 100, 1900)]:
        assert (oracle.cpu_dottt(g.n, g.src, g.dst, g.t, *d) == oracle.count(g.n, g.src, g.dst, g.t, *d)).all()
    g = synth.plain_tiny()
    for x in (0, 10**4, 10**5, 10**6):
        assert (oracle.cpu_dottt(g.n, g.src, g.dst, g.t, x, x, x) == oracle.count(g.n, g.src, g.dst, g.t, x, x, x)).all()


def test_infinite_delta_identity_and_relabelling():
    for seed in range(6):
        g = synth.tiny_multigraph(seed, n=10, m=120, t_range=30)
        inf = 10**12
        got = oracle.cpu_dottt(g.n, g.src, g.dst, g.t, inf, inf, inf)
        st = oracle.stats(g.n, g.src, g.dst, g.t)
        assert int(got.sum()) == st["sum_sigma3"], seed
        perm = np.random.default_rng(seed).permutation(g.n).astype(np.uint32)
        for d in [(5, 3, 4), (12, 12, 12)]:
            a = oracle.cpu_dottt(g.n, g.src, g.dst, g.t, *d)
            b = oracle.cpu_dottt(g.n, perm[g.src], perm[g.dst], g.t, *d)
            assert (a == b).all(), (seed, d)


def test_invalid_arguments():
    g = synth.seed_graph()
    with pytest.raises(oracle.OracleError):
        oracle.cpu_dottt(g.n, g.src, g.dst, g.t, -1, 0, 0)
    with pytest.raises(oracle.OracleError):
        oracle.cpu_dottt(g.n, g.src, g.dst, g.t, 1, 1, 1, 5, 4)
    assert (oracle.cpu_dottt(g.n, g.src[:0], g.dst[:0], g.t[:0], 1, 1, 1) == 0).all()
