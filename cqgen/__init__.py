"""Seeded synthetic inputs: LFR-style graphs, partition perturbations and edge weights.

This package only generates inputs (a symmetric int32 CSR graph, ground-truth
labels, perturbed labels and symmetric float32 edge weights).  It holds none of the arithmetic of the metrics:
both the GPU library and the CPU oracle consume what it produces.
"""
from .lfr import LFRParams, LFRGraph, lfr_graph, perturb_labels, random_labels, CONFIGS  # noqa: F401
from .smallgraphs import (  # noqa: F401
    csr_from_edges, cliques_graph, complete_graph, erdos_renyi, star_graph, ring_graph,
)
from .weights import edge_weights  # noqa: F401
