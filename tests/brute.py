"""Exhaustive checks that pin the oracle, written independently of it (pure Python, tiny inputs).

- brute_force(): every C(m,3) triple of kept edges, ordered by the key (t, input index), tested
  against Definition 1's three inequalities, and classified through the paper's own Table 2 by
  reading its temporal ordering (Figure 3) and orientation (Figure 4) relative to u < v < w.
  The oracle classifies with Figure 2 directly, so agreement ties Table 2 and Figure 2 together.
- lemma1_cells(): Lemma 1's double sum for every static triangle and (pi, rho) cell, for inputs
  with distinct timestamps (the setting in which the lemma is stated).
"""
from __future__ import annotations

import itertools

import numpy as np

from paper_tables import fig3_orders, fig4_orientations, table2_psi

INT64_MIN = -(1 << 63)
INT64_MAX = (1 << 63) - 1

_PI = {v: k for k, v in fig3_orders().items()}            # (p1, p2, p3) -> pi
_RHO = {}
for _k, _d in fig4_orientations().items():
    _RHO[tuple(_d[p] == tuple(p) for p in ("uv", "uw", "vw"))] = _k   # forward flags -> rho
_PSI = table2_psi()


def _kept(src, dst, t, t_lo, t_hi):
    return [i for i in range(len(src))
            if int(src[i]) != int(dst[i]) and t_lo <= int(t[i]) <= t_hi]


def _cell_of(edges):
    """(pi, rho) of three edges (src, dst) listed in temporal order, forming a triangle."""
    verts = sorted({x for e in edges for x in e})
    u, v, w = verts
    name = {frozenset((u, v)): "uv", frozenset((u, w)): "uw", frozenset((v, w)): "vw"}
    names = tuple(name[frozenset(e)] for e in edges)
    fwd = {}
    for e, p in zip(edges, names):
        lo = {"uv": u, "uw": u, "vw": v}[p]
        fwd[p] = e[0] == lo
    pi = _PI[names]
    rho = _RHO[(fwd["uv"], fwd["uw"], fwd["vw"])]
    return pi, rho


def brute_force(src, dst, t, d13, d12, d23, t_lo=INT64_MIN, t_hi=INT64_MAX):
    """(types int64[8], cells int64[6, 8]) by exhaustive enumeration of edge triples."""
    keep = _kept(src, dst, t, t_lo, t_hi)
    types = np.zeros(8, dtype=np.int64)
    cells = np.zeros((6, 8), dtype=np.int64)
    for tri in itertools.combinations(keep, 3):
        pairs = [frozenset((int(src[i]), int(dst[i]))) for i in tri]
        if len(set(pairs)) != 3 or len(frozenset().union(*pairs)) != 3:
            continue
        e1, e2, e3 = sorted(tri, key=lambda i: (int(t[i]), i))
        t1, t2, t3 = int(t[e1]), int(t[e2]), int(t[e3])
        if t2 - t1 > d12 or t3 - t2 > d23 or t3 - t1 > d13:
            continue
        pi, rho = _cell_of([(int(src[i]), int(dst[i])) for i in (e1, e2, e3)])
        types[_PSI[pi][rho] - 1] += 1
        cells[pi - 1, rho - 1] += 1
    return types, cells


def lemma1_cells(src, dst, t, d13, d12, d23):
    """Lemma 1 (Section 4) summed over every static triangle, per (pi, rho) cell.

    For each triangle u < v < w, ordering pi and orientation rho: S_i are the edges on pair pi(i) in
    direction rho(pi(i)); the count is the sum over e2 in S2 and e1 in S1 with
    t(e1) in [t(e2) - d12, t(e2)] of EC([t(e2), min(t(e2) + d23, t(e1) + d13)], S3).
    Assumes distinct timestamps, as the lemma does.
    """
    keep = _kept(src, dst, t, INT64_MIN, INT64_MAX)
    by_pair = {}
    for i in keep:
        a, b = int(src[i]), int(dst[i])
        by_pair.setdefault(frozenset((a, b)), []).append(i)
    verts = sorted({x for p in by_pair for x in p})
    cells = np.zeros((6, 8), dtype=np.int64)
    orders = fig3_orders()
    orients = fig4_orientations()
    for u, v, w in itertools.combinations(verts, 3):
        P = {"uv": frozenset((u, v)), "uw": frozenset((u, w)), "vw": frozenset((v, w))}
        if not all(p in by_pair for p in P.values()):
            continue
        names = {"u": u, "v": v, "w": w}
        for pi, seq in orders.items():
            for rho, dirs in orients.items():
                S = []
                for p in seq:
                    tail = names[dirs[p][0]]
                    S.append(sorted(int(t[i]) for i in by_pair[P[p]] if int(src[i]) == tail))
                S1, S2, S3 = S
                total = 0
                for t2 in S2:
                    for t1 in S1:
                        if t2 - d12 <= t1 <= t2:
                            hi = min(t2 + d23, t1 + d13)
                            total += sum(1 for t3 in S3 if t2 <= t3 <= hi)
                cells[pi - 1, rho - 1] += total
    return cells


def sum_sigma3(src, dst, t):
    """Sum over static triangles of the product of the three pair multiplicities."""
    keep = _kept(src, dst, t, INT64_MIN, INT64_MAX)
    mult = {}
    for i in keep:
        p = frozenset((int(src[i]), int(dst[i])))
        mult[p] = mult.get(p, 0) + 1
    verts = sorted({x for p in mult for x in p})
    s = 0
    for u, v, w in itertools.combinations(verts, 3):
        a, b, c = frozenset((u, v)), frozenset((u, w)), frozenset((v, w))
        if a in mult and b in mult and c in mult:
            s += mult[a] * mult[b] * mult[c]
    return s
