"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle scripts.

This package only produces arrays (arcs, weights, held-out pairs, negative pairs for
evaluation).  It holds none of the embedding method's arithmetic: no alias tables, no
sampling of training tuples, no SGD.  Both the CPU oracle and the GPU library are fed
from here, and neither one imports the other.
"""
from .graphs import (  # noqa: F401
    Graph,
    rmat_graph,
    config_graph,
    holdout_split,
    auc_negatives,
    batch_graph_specs,
    batch_graph,
    small_batch,
    mid_graph,
    CONFIGS,
)
