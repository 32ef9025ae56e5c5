"""Readers for the fixtures under tests/golden/, transcribed from the paper's Figures 2-4 and
Table 2.  Used by the tests only."""
from __future__ import annotations

import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def fig2_types():
    """{k: [(tail, head) at position 1, 2, 3]} over vertex names 'a', 'b', 'c' (Figure 2)."""
    out = {}
    for row in _rows("fig2_types.txt"):
        out[int(row[0][1:])] = [tuple(e.split(">")) for e in row[1:4]]
    return out


def fig3_orders():
    """{pi: (pair at position 1, 2, 3)} with pairs named 'uv', 'uw', 'vw' (Figure 3)."""
    return {int(r[0][2:]): tuple(r[1:4]) for r in _rows("fig3_orders.txt")}


def fig4_orientations():
    """{rho: {'uv': (tail, head), 'uw': ..., 'vw': ...}} (Figure 4)."""
    out = {}
    for r in _rows("fig4_orientations.txt"):
        out[int(r[0][3:])] = {p: tuple(e.split(">")) for p, e in zip(("uv", "uw", "vw"), r[1:4])}
    return out


def table2_psi():
    """psi[pi][rho] -> type, all 1-based (Table 2)."""
    return {int(r[0][2:]): {j + 1: int(x) for j, x in enumerate(r[1:9])} for r in _rows("table2_psi.txt")}
