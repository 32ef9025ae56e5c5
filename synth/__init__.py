"""Seeded synthetic temporal multigraphs shared by the tests, the benchmark and the oracle checks.

This package draws random numbers and shapes workloads; it holds none of the counting
arithmetic of the method.
"""
from .graphs import (  # noqa: F401
    TemporalGraph,
    SEED_BASE,
    tiny_multigraph,
    seed_graph,
    plain_tiny,
    plain_medium,
    plain_full,
    batch_graph,
    batch_delta,
    served_stream,
    delta_triple_like_batch,
    clique_graph,
    contested_graph,
    long_lists_graph,
    replicated,
    disjoint_union,
)
