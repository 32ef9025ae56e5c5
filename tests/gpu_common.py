"""Helpers shared by the GPU tests: a per-session context and graph construction through the
C ABI, printing the case name before each device step so that a failing run names it."""
from __future__ import annotations

import sys

import numpy as np

import paper_2106_02762_amd as dt

INF = dt.DT_INF


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


class Built:
    """A loaded and built graph with its host arrays."""

    def __init__(self, ctx, g, name, path=0):
        self.ctx = ctx
        self.n, self.src, self.dst, self.t = g.n, g.src, g.dst, g.t
        self.name = name
        say("load+build", name, "n", g.n, "m", g.m)
        self.h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
        dt.dt_graph_build(self.h)
        if path:
            say("force path", path)
            dt.dt_graph_set_tuning(self.h, force_path=path)

    def count(self, d13, d12, d23, t_lo=dt.INT64_MIN, t_hi=INF):
        say("count", self.name, d13, d12, d23, t_lo, t_hi)
        return dt.dt_count(self.h, d13, d12, d23, t_lo, t_hi)

    def free(self):
        dt.dt_graph_free(self.h)
