"""Non-box test workloads shared by the oracle pins and the library's host
and GPU checks (problem descriptions only)."""

import numpy as np

from workloads.gen import partition_workload
from workloads.partition import grown_groups, grown_partition, kd_partition


def ring_2d():
    """8 x 6 Q1 elements in 2x2-element blocks, whole boundary clamped; block
    rows (bottom to top) A A A A / Y B X A / A A A A with A = 0, B = 1, X = 2,
    Y = 3: A wraps B, X and Y, so A and B touch in two separate patches (above
    and below B), as do A and Y, and A, B with Y or X meet at single nodes
    above and below."""
    blocks = np.array([[0, 0, 0, 0], [3, 1, 2, 0], [0, 0, 0, 0]])   # [by, bx]
    e = np.arange(48)
    part = blocks[(e // 8) // 2, (e % 8) // 2]
    return partition_workload("ring", "poisson", (8, 6), part, dirichlet="all", constraints="c")


def nonbox(kind, L, n=12, parts=27, groups=4, seed=1):
    """3D elasticity on n^3 elements, E = 10^(2U) (default_rng(8)), divided
    into `parts` subdomains by k-d bisection ("kd") or graph growing
    ("grown"); at L = 3 the subdomains are grown into `groups` groups."""
    n_el = (n, n, n)
    part = kd_partition(n_el, parts, seed) if kind == "kd" else grown_partition(n_el, parts, seed)
    parents = [grown_groups(n_el, part, groups, seed)] if L == 3 else []
    young = 10 ** (2 * np.random.default_rng(8).random(n ** 3))
    return partition_workload(f"{kind}_L{L}", "elasticity", n_el, part, parents, young=young)
