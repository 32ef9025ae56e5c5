"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU needed).

Each check is chosen so that a plausible slip in the oracle (a wrong type in the classifier, a
swapped delta, an off-by-one at a delta boundary, a mishandled tie or window) fails at least one:
- Figure 2's eight panels, each a unit vector, with every delta boundary probed by +-1;
- Table 2 against the oracle's own Figure-2 classifier and Figure 3/4 cell decoding, all 48 cells;
- exhaustive brute force over all edge triples (classified through Table 2) on random multigraphs
  with many equal timestamps and self-loops, and on the 50-node / 300-edge seed graph;
- Lemma 1's double sum per cell on graphs with distinct timestamps;
- delta = infinity: the type counts sum to the sum over static triangles of the product of the
  three pair multiplicities;
- monotonicity in each delta, invariance under node relabelling, the type permutations under edge
  reversal and time reversal (derived from Figure 2), and windows equal to filtering.
"""
import itertools

import numpy as np
import pytest

import synth
from brute import brute_force, lemma1_cells, sum_sigma3
from paper_tables import fig2_types, fig3_orders, fig4_orientations, table2_psi

INF = (1 << 63) - 1


def _graph_from(edges, times):
    src = np.array([e[0] for e in edges], dtype=np.uint32)
    dst = np.array([e[1] for e in edges], dtype=np.uint32)
    return src, dst, np.array(times, dtype=np.int64)


@pytest.mark.parametrize("k", range(1, 9))
def test_fig2_panel_is_unit_vector(oracle_mod, k):
    panel = fig2_types()[k]
    for perm in itertools.permutations(range(3)):
        name = dict(zip("abc", perm))
        edges = [(name[x], name[y]) for x, y in panel]
        src, dst, t = _graph_from(edges, [1, 2, 3])
        got = oracle_mod.count(3, src, dst, t, 2, 1, 1)
        want = np.zeros(8, dtype=np.int64)
        want[k - 1] = 1
        assert (got == want).all(), (k, perm, got)


@pytest.mark.parametrize("k", [1, 4, 5, 8])
def test_fig2_delta_boundaries(oracle_mod, k):
    """Definition 1 uses <= on every gap: a gap equal to its delta counts, one more does not."""
    panel = fig2_types()[k]
    src, dst, _ = _graph_from([({"a": 0, "b": 1, "c": 2}[x], {"a": 0, "b": 1, "c": 2}[y])
                               for x, y in panel], [0, 0, 0])
    for t1, t2, t3 in [(10, 14, 20), (0, 7, 9), (5, 5 + 3, 5 + 3 + 6)]:
        t = np.array([t1, t2, t3], dtype=np.int64)
        g12, g23, g13 = t2 - t1, t3 - t2, t3 - t1
        for d12, d23, d13 in [(g12, g23, g13), (g12 - 1, g23, g13), (g12, g23 - 1, g13),
                              (g12, g23, g13 - 1), (g12 + 5, g23 + 5, g13 + 5)]:
            got = oracle_mod.count(3, src, dst, t, d13, d12, d23)
            ok = g12 <= d12 and g23 <= d23 and g13 <= d13
            assert int(got.sum()) == int(ok) and int(got[k - 1]) == int(ok), (t, d12, d23, d13, got)


def test_table2_matches_oracle_classifier_and_cells(oracle_mod):
    psi = table2_psi()
    orders = fig3_orders()
    orients = fig4_orientations()
    name = {"u": 0, "v": 1, "w": 2}
    seen = np.zeros(9, dtype=int)
    for pi, seq in orders.items():
        for rho, dirs in orients.items():
            edges = [(name[dirs[p][0]], name[dirs[p][1]]) for p in seq]
            src, dst, t = _graph_from(edges, [1, 2, 3])
            ty, ce = oracle_mod.count(3, src, dst, t, 10, 10, 10, cells=True)
            want_t = np.zeros(8, dtype=np.int64)
            want_t[psi[pi][rho] - 1] = 1
            want_c = np.zeros((6, 8), dtype=np.int64)
            want_c[pi - 1, rho - 1] = 1
            assert (ty == want_t).all(), (pi, rho, ty)
            assert (ce == want_c).all(), (pi, rho)
            seen[psi[pi][rho]] += 1
    assert (seen[1:] == 6).all()


def _delta_grid(rng, tr):
    out = [(INF, INF, INF), (0, 0, 0)]
    for _ in range(6):
        out.append(tuple(int(x) for x in rng.integers(0, tr + 2, 3)))
    return out


@pytest.mark.parametrize("seed", range(40))
def test_oracle_equals_brute_force_tiny(oracle_mod, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 7))
    m = int(rng.integers(3, 15))
    tr = int(rng.integers(1, 8))
    g = synth.tiny_multigraph(seed, n=n, m=m, t_range=tr)
    for d13, d12, d23 in _delta_grid(rng, tr):
        lo, hi = (-INF - 1, INF) if rng.random() < 0.6 else sorted(int(x) for x in rng.integers(0, tr, 2))
        bt, bc = brute_force(g.src, g.dst, g.t, d13, d12, d23, lo, hi)
        ot, oc = oracle_mod.count(g.n, g.src, g.dst, g.t, d13, d12, d23, lo, hi, cells=True)
        assert (ot == bt).all(), (seed, d13, d12, d23, lo, hi, ot, bt)
        assert (oc == bc).all(), (seed, d13, d12, d23, lo, hi)


@pytest.mark.slow
def test_oracle_equals_brute_force_seed_graph(oracle_mod):
    g = synth.seed_graph()
    for d13, d12, d23 in [(300, 200, 150), (INF, INF, INF), (50, 50, 50)]:
        bt, bc = brute_force(g.src, g.dst, g.t, d13, d12, d23)
        ot, oc = oracle_mod.count(g.n, g.src, g.dst, g.t, d13, d12, d23, cells=True)
        assert (ot == bt).all() and (oc == bc).all(), (d13, d12, d23, ot, bt)


@pytest.mark.parametrize("seed", range(12))
def test_oracle_cells_equal_lemma1(oracle_mod, seed):
    rng = np.random.default_rng(2000 + seed)
    g = synth.tiny_multigraph(seed + 500, n=5, m=14, t_range=10**6)
    assert np.unique(g.t).shape[0] == g.m  # Lemma 1 is stated for distinct timestamps
    for _ in range(4):
        d13, d12, d23 = (int(x) for x in rng.integers(0, 10**6, 3))
        _, oc = oracle_mod.count(g.n, g.src, g.dst, g.t, d13, d12, d23, cells=True)
        assert (oc == lemma1_cells(g.src, g.dst, g.t, d13, d12, d23)).all()


@pytest.mark.parametrize("seed", range(10))
def test_infinite_delta_product_identity(oracle_mod, seed):
    g = synth.tiny_multigraph(seed + 900, n=7, m=25, t_range=5)
    ty, ce = oracle_mod.count(g.n, g.src, g.dst, g.t, INF, INF, INF, cells=True)
    s3 = sum_sigma3(g.src, g.dst, g.t)
    assert int(ty.sum()) == s3
    st = oracle_mod.stats(g.n, g.src, g.dst, g.t)
    assert st["sum_sigma3"] == s3
    # per orientation: the six orderings of one rho cover every triple of that orientation once
    assert int(ce.sum()) == s3


def test_infinite_delta_product_identity_tiny_workload(oracle_mod):
    g = synth.plain_tiny()
    ty = oracle_mod.count(g.n, g.src, g.dst, g.t, INF, INF, INF)
    st = oracle_mod.stats(g.n, g.src, g.dst, g.t)
    assert int(ty.sum()) == st["sum_sigma3"] > 0


@pytest.mark.parametrize("seed", range(6))
def test_monotone_in_each_delta(oracle_mod, seed):
    g = synth.tiny_multigraph(seed + 40, n=6, m=30, t_range=20)
    base = (6, 4, 4)
    ref = oracle_mod.count(g.n, g.src, g.dst, g.t, *base)
    for j in range(3):
        prev = ref
        for inc in range(1, 8):
            d = list(base)
            d[j] += inc
            cur = oracle_mod.count(g.n, g.src, g.dst, g.t, *d)
            assert (cur >= prev).all()
            prev = cur


@pytest.mark.parametrize("seed", range(6))
def test_relabel_invariance(oracle_mod, seed):
    g = synth.tiny_multigraph(seed + 70, n=8, m=40, t_range=6)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(g.n).astype(np.uint32)
    for d in [(3, 2, 2), (INF, INF, INF), (1, 1, 0)]:
        a = oracle_mod.count(g.n, g.src, g.dst, g.t, *d)
        b = oracle_mod.count(g.n, perm[g.src], perm[g.dst], g.t, *d)
        assert (a == b).all()


# Type permutations derived from Figure 2 (0-based type indices).
_REVERSE_EDGES = [4, 6, 5, 7, 0, 2, 1, 3]   # (T1 T5)(T2 T7)(T3 T6)(T4 T8)
_REVERSE_TIME = [2, 6, 0, 7, 5, 4, 1, 3]    # (T1 T3)(T2 T7)(T4 T8)(T5 T6)


@pytest.mark.parametrize("seed", range(8))
def test_edge_reversal_permutes_types(oracle_mod, seed):
    g = synth.tiny_multigraph(seed + 110, n=6, m=30, t_range=8)
    for d in [(5, 3, 2), (INF, INF, INF), (4, 4, 1)]:
        a = oracle_mod.count(g.n, g.src, g.dst, g.t, *d)
        b = oracle_mod.count(g.n, g.dst, g.src, g.t, *d)
        assert (b == a[_REVERSE_EDGES]).all()


@pytest.mark.parametrize("seed", range(8))
def test_time_reversal_permutes_types(oracle_mod, seed):
    g = synth.tiny_multigraph(seed + 150, n=6, m=30, t_range=8)
    r = slice(None, None, -1)  # reversed input order reverses the tie-break as well
    for d13, d12, d23 in [(5, 3, 2), (INF, INF, INF), (4, 4, 1), (6, 1, 5)]:
        a = oracle_mod.count(g.n, g.src, g.dst, g.t, d13, d12, d23, 1, 6)
        b = oracle_mod.count(g.n, g.src[r], g.dst[r], -g.t[r], d13, d23, d12, -6, -1)
        assert (b == a[_REVERSE_TIME]).all()


@pytest.mark.parametrize("seed", range(6))
def test_window_equals_filter(oracle_mod, seed):
    g = synth.tiny_multigraph(seed + 190, n=7, m=40, t_range=30)
    for lo, hi in [(5, 20), (0, 0), (29, 29), (-5, 100), (12, 11 + 7)]:
        keep = (g.t >= lo) & (g.t <= hi)
        a = oracle_mod.count(g.n, g.src, g.dst, g.t, 6, 4, 3, lo, hi)
        b = oracle_mod.count(g.n, g.src[keep], g.dst[keep], g.t[keep], 6, 4, 3)
        assert (a == b).all()


def test_errors(oracle_mod):
    src, dst, t = _graph_from([(0, 1), (1, 2)], [1, 2])
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.count(2, src, dst, t, 1, 1, 1)            # node id >= n
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.count(3, src, dst, t, -1, 1, 1)           # negative delta
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.count(3, src, dst, t, 1, 1, 1, 5, 4)      # empty window bounds


def test_empty_and_degenerate_inputs(oracle_mod):
    e = np.zeros(0, dtype=np.uint32)
    assert (oracle_mod.count(5, e, e, np.zeros(0, np.int64), 1, 1, 1) == 0).all()
    src, dst, t = _graph_from([(0, 0), (1, 1), (2, 2)], [1, 2, 3])   # self-loops only
    assert (oracle_mod.count(3, src, dst, t, INF, INF, INF) == 0).all()
    st = oracle_mod.stats(3, src, dst, t)
    assert st["self_loops"] == 3 and st["m_static"] == 0


def test_stats_and_core_numbers(oracle_mod):
    # K4 plus a pendant path: core numbers 3,3,3,3,1,1; one multi-edge pair of multiplicity 3
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (3, 4), (4, 5), (1, 0), (0, 1)]
    src, dst, t = _graph_from(edges, list(range(len(edges))))
    st, core = oracle_mod.stats(6, src, dst, t, core=True)
    assert list(core) == [3, 3, 3, 3, 1, 1]
    assert st["degeneracy"] == 3 and st["n_triangles"] == 4 and st["m_static"] == 8
    assert st["max_multiplicity"] == 3
    assert st["sum_sigma3"] == 3 + 3 + 1 + 1  # triangles 012 and 013 contain pair 01 (x3)
    tri = oracle_mod.triangles(6, src, dst, t)
    assert tri.tolist() == [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]
