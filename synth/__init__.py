"""Seeded synthetic inputs for the PilotANN GPU-stage workloads.

This package only *draws* inputs: base vectors, queries, the random orders
that the sampling and entry-selection steps consume, and the proximity-graph
fixtures that play the role of the externally trained graph index (the paper
reuses the graph FAISS built; it does not construct one itself).  It holds
none of PilotANN's own arithmetic (projection, sampling rule, entry
selection, traversal, refinement).  Both the library path and the oracle
take their inputs from here.
"""

from .data import (  # noqa: F401
    WorkloadSpec,
    SPECS,
    make_rng,
    gmm_centers,
    nested_centers,
    gmm_points,
    anisotropic_points,
    base_vectors,
    query_vectors,
    node_order,
    pivot_choice,
    kmeans_init_choice,
)
