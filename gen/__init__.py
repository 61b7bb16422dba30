"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Nothing in this package implements any step of the mapping method."""
from .graphs import (Graph, from_edges, grid2d, path_graph, random_balanced_mapping,
                     random_mapping, rgg, rmat, rmat_n, shuffle_rows)
from .workloads import (WORKLOADS, Instance, Workload, batch_member, batch_members,
                        batch_spec, get, instance, serve_arrivals, serve_pool_spec,
                        serve_requests, serve_stream)

__all__ = ["Graph", "from_edges", "grid2d", "path_graph", "rgg", "rmat",
           "random_balanced_mapping", "random_mapping", "shuffle_rows",
           "rmat_n", "WORKLOADS", "Workload", "get", "Instance", "instance",
           "batch_member", "batch_members", "batch_spec", "serve_arrivals",
           "serve_pool_spec", "serve_requests", "serve_stream"]
