"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package holds graph and query generators and the CSR canonicaliser only.
It contains none of the estimator's arithmetic: no probes, no walks, no
planner. Both the CPU oracle (through the tests) and the HIP library consume
what it produces; neither imports the other.
"""

from .graphs import (  # noqa: F401
    Csr,
    barabasi_albert,
    chung_lu,
    grid_minus_edges,
    complete_graph,
    cycle_graph,
    path_graph,
    random_connected,
    csr_from_edges,
    largest_component,
    workload_graph,
    WORKLOADS,
)
from .queries import uniform_pairs, mixed_eps_L  # noqa: F401
