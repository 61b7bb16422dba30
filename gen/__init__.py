"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Nothing in this package implements any step of the mapping method."""
from .graphs import (Graph, from_edges, grid2d, path_graph, random_balanced_mapping,
                     random_mapping, rgg, rmat, shuffle_rows)
from .workloads import WORKLOADS, Workload, get

__all__ = ["Graph", "from_edges", "grid2d", "path_graph", "rgg", "rmat",
           "random_balanced_mapping", "random_mapping", "shuffle_rows",
           "WORKLOADS", "Workload", "get"]
