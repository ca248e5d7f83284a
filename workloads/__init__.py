"""Seeded synthetic problem generators shared by the oracle, the tests and the bench.

This package only describes *problems*: structured meshes, Dirichlet node sets,
box partitions, level groupings and seeded material fields.  It holds none of
the domain-decomposition arithmetic (no element matrices, no assembly, no
interface or coarse-space logic); both the CPU oracle and the GPU library
derive everything else from these arrays independently.
"""

from .gen import (  # noqa: F401
    Workload,
    structured_mesh,
    box_partition,
    group_parents,
    random_cuts,
    box_workload,
    config,
    large_subdomains,
    CONFIG_NAMES,
)
