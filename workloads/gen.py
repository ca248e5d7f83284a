"""Structured-mesh workloads with box partitions (problem descriptions only).

Conventions (shared *definitions*, not shared arithmetic):

* The domain is the unit square/cube, split into ``n_el[d]`` equal elements per
  axis, element size ``h = 1 / n_el[0]`` (all axes equal in every workload).
* Nodes are numbered lexicographically with x fastest:
  ``node(i, j[, k]) = i + (nx+1) * (j + (ny+1) * k)``.
* Elements likewise: ``elem(a, b[, c]) = a + nx * (b + ny * c)``.
* Local node order of a quadrilateral is counter-clockwise
  ``(0,0), (1,0), (1,1), (0,1)``; of a hexahedron the bottom face
  counter-clockwise then the top face: ``(0,0,0), (1,0,0), (1,1,0), (0,1,0),
  (0,0,1), (1,0,1), (1,1,1), (0,1,1)``.
* A DOF is ``node * ndof + component``.  Dirichlet conditions are homogeneous
  and act on every component of a listed node.
* Boxes (level-1 subdomains) are numbered lexicographically with x fastest over
  the box grid given by per-axis cut lists; level-l subdomains group boxes of
  level l-1 in the same way.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np


@dataclass
class Workload:
    name: str
    physics: str                 # "poisson" (1 DOF/node) or "elasticity" (3 DOF/node)
    dim: int
    n_el: Tuple[int, ...]        # elements per axis
    elem_nodes: np.ndarray       # int32 [n_elems, 2**dim]
    dirichlet_nodes: np.ndarray  # bool  [n_nodes]
    young: np.ndarray            # float64 [n_elems], per-element modulus E_e
    poisson_ratio: float
    body_force: Tuple[float, ...]
    cuts: List[np.ndarray]       # per-axis element indices of box boundaries
    elem_to_sub: np.ndarray      # int32 [n_elems]
    sub_to_parent: List[np.ndarray] = field(default_factory=list)  # levels 2..L-1
    constraints: str = "cef"     # "c" corners only, "cef" corners+edges+faces
    n_levels: int = 2
    seed: int = 0

    @property
    def ndof(self) -> int:
        return 1 if self.physics == "poisson" else self.dim

    @property
    def h(self) -> float:
        return 1.0 / self.n_el[0]

    @property
    def n_nodes(self) -> int:
        return int(np.prod([n + 1 for n in self.n_el]))

    @property
    def n_elems(self) -> int:
        return int(np.prod(self.n_el))

    @property
    def n_subdomains(self) -> int:
        return int(self.elem_to_sub.max()) + 1


def structured_mesh(n_el: Sequence[int]) -> np.ndarray:
    """Element-to-node connectivity of a structured quad/hex mesh."""
    dim = len(n_el)
    if dim == 2:
        nx, ny = n_el
        a, b = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
        a = a.ravel(); b = b.ravel()
        n0 = a + (nx + 1) * b
        return np.stack([n0, n0 + 1, n0 + 1 + (nx + 1), n0 + (nx + 1)], axis=1).astype(np.int32)
    if dim == 3:
        nx, ny, nz = n_el
        c, b, a = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        a = a.ravel(); b = b.ravel(); c = c.ravel()
        sx, sy = 1, nx + 1
        sz = (nx + 1) * (ny + 1)
        n0 = a * sx + b * sy + c * sz
        bottom = [n0, n0 + sx, n0 + sx + sy, n0 + sy]
        top = [q + sz for q in bottom]
        return np.stack(bottom + top, axis=1).astype(np.int32)
    raise ValueError("dim must be 2 or 3")


def _node_grid(n_el: Sequence[int]) -> List[np.ndarray]:
    """Integer coordinates of every node (lexicographic, x fastest)."""
    axes = [np.arange(n + 1) for n in n_el]
    grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
    return [g.ravel() for g in grids]


def box_partition(n_el: Sequence[int], cuts: Sequence[Sequence[int]]) -> np.ndarray:
    """Element -> box id for a tensor grid of boxes given by per-axis cut lists."""
    dim = len(n_el)
    elem_axes = [np.arange(n) for n in n_el]
    box_of_axis = []
    for d in range(dim):
        c = np.asarray(cuts[d])
        if c[0] != 0 or c[-1] != n_el[d] or np.any(np.diff(c) <= 0):
            raise ValueError(f"bad cut list on axis {d}: {c}")
        box_of_axis.append(np.searchsorted(c, elem_axes[d], side="right") - 1)
    grids = np.meshgrid(*box_of_axis[::-1], indexing="ij")[::-1]
    nb = [len(c) - 1 for c in cuts]
    box = np.zeros_like(grids[0])
    stride = 1
    for d in range(dim):
        box = box + grids[d] * stride
        stride *= nb[d]
    return box.ravel().astype(np.int32)


def group_parents(n_boxes: Sequence[int], group: Sequence[int]) -> Tuple[np.ndarray, Tuple[int, ...]]:
    """Parent id of each box when boxes are grouped ``group[d]`` at a time per axis."""
    dim = len(n_boxes)
    for d in range(dim):
        if n_boxes[d] % group[d]:
            raise ValueError("group size must divide the box count on every axis")
    parent_dims = tuple(n_boxes[d] // group[d] for d in range(dim))
    idx = np.arange(int(np.prod(n_boxes)))
    coords = []
    rem = idx.copy()
    for d in range(dim):
        coords.append(rem % n_boxes[d])
        rem //= n_boxes[d]
    parent = np.zeros_like(idx)
    stride = 1
    for d in range(dim):
        parent += (coords[d] // group[d]) * stride
        stride *= parent_dims[d]
    return parent.astype(np.int32), parent_dims


def random_cuts(seed: int, n: int = 80, parts: int = 8, lo: int = 4, hi: int = 16, dim: int = 3) -> List[np.ndarray]:
    """Random axis-aligned full cutting planes: per axis (x, y, z in order) draw
    ``parts`` box widths in [lo, hi] from one generator until they sum to ``n``."""
    rng = np.random.default_rng(seed)
    cuts = []
    for _ in range(dim):
        while True:
            widths = rng.integers(lo, hi + 1, parts)
            if widths.sum() == n:
                break
        cuts.append(np.concatenate([[0], np.cumsum(widths)]).astype(np.int64))
    return cuts


def partition_workload(
    name: str,
    physics: str,
    n_el: Sequence[int],
    elem_to_sub: np.ndarray,
    sub_to_parent: Sequence[np.ndarray] = (),
    young: np.ndarray | None = None,
    poisson_ratio: float = 0.3,
    body_force: Sequence[float] | None = None,
    dirichlet: str = "x0",
    constraints: str = "cef",
    seed: int = 0,
    cuts: Sequence[Sequence[int]] = (),
) -> Workload:
    """Workload on the structured mesh with any division: ``elem_to_sub`` for
    level 1 and ``sub_to_parent`` for levels 2..L-1 (L = len + 2).
    ``dirichlet`` is "x0" (face x = 0 clamped) or "all" (whole boundary)."""
    dim = len(n_el)
    n_el = tuple(int(n) for n in n_el)
    elem_nodes = structured_mesh(n_el)
    coords = _node_grid(n_el)
    if dirichlet == "x0":
        dir_nodes = coords[0] == 0
    elif dirichlet == "all":
        dir_nodes = np.zeros(coords[0].shape, dtype=bool)
        for d in range(dim):
            dir_nodes |= (coords[d] == 0) | (coords[d] == n_el[d])
    else:
        raise ValueError(dirichlet)
    n_elems = int(np.prod(n_el))
    if young is None:
        young = np.ones(n_elems)
    if body_force is None:
        body_force = (1.0,) if physics == "poisson" else tuple([0.0] * (dim - 1) + [-1.0])
    return Workload(
        name=name, physics=physics, dim=dim, n_el=n_el, elem_nodes=elem_nodes,
        dirichlet_nodes=dir_nodes, young=np.asarray(young, dtype=np.float64),
        poisson_ratio=poisson_ratio, body_force=tuple(body_force), cuts=[np.asarray(c, dtype=np.int64) for c in cuts],
        elem_to_sub=np.asarray(elem_to_sub, dtype=np.int32),
        sub_to_parent=[np.asarray(p, dtype=np.int32) for p in sub_to_parent], constraints=constraints,
        n_levels=len(sub_to_parent) + 2, seed=seed,
    )


def box_workload(
    name: str,
    physics: str,
    n_el: Sequence[int],
    cuts: Sequence[Sequence[int]],
    groups: Sequence[Sequence[int]] = (),
    young: np.ndarray | None = None,
    poisson_ratio: float = 0.3,
    body_force: Sequence[float] | None = None,
    dirichlet: str = "x0",
    constraints: str = "cef",
    seed: int = 0,
) -> Workload:
    """General box-partitioned workload.

    ``groups`` lists, for levels 2..L-1, how many level-(l-1) subdomains per axis
    form one level-l subdomain; the number of levels is ``len(groups) + 2``.
    ``dirichlet`` is "x0" (face x = 0 clamped) or "all" (whole boundary).
    """
    cuts = [np.asarray(c, dtype=np.int64) for c in cuts]
    elem_to_sub = box_partition(n_el, cuts)
    n_boxes = tuple(len(c) - 1 for c in cuts)
    parents = []
    cur = n_boxes
    for g in groups:
        p, cur = group_parents(cur, g)
        parents.append(p)
    return partition_workload(name, physics, n_el, elem_to_sub, parents, young=young, poisson_ratio=poisson_ratio,
                              body_force=body_force, dirichlet=dirichlet, constraints=constraints, seed=seed,
                              cuts=cuts)


def uniform_cuts(n: int, parts: int) -> np.ndarray:
    if n % parts:
        raise ValueError("parts must divide n")
    return np.arange(0, n + 1, n // parts)


def large_subdomains(n: int = 40, parts: int = 2, seed: int = 3) -> Workload:
    """Subdomains of (n/parts)^3 elements (20^3 by default: 27,783 DOFs each,
    the tens of thousands of unknowns per subdomain of the paper's runs):
    3D elasticity on n^3 elements, parts^3 box subdomains, 2 levels,
    E = 10^(2U), U ~ U(0,1) from default_rng(seed)."""
    young = 10.0 ** (2.0 * np.random.default_rng(seed).random(n ** 3))
    sub = n // parts
    return box_workload(f"elasticity3d_{n}cube_{parts ** 3}sub{sub}_L2", "elasticity", (n,) * 3,
                        [uniform_cuts(n, parts)] * 3, young=young, seed=seed)


CONFIG_NAMES = {
    1: "poisson2d_32x32_4x4sub_L2",
    2: "elasticity3d_48cube_64sub",
    3: "elasticity3d_96cube_1728sub",
    4: "elasticity3d_80cube_512uneven_L3",
    5: "elasticity3d_64cube_512sub_L3_grad",
    6: "elasticity3d_40cube_8sub20_L2",
}


def config(k: int, levels: int | None = None, seed: int = 0) -> Workload:
    """The benchmark workloads, numbered 1..6.

    1. 2D Poisson -Lap u = 1, 32x32 Q1, Dirichlet everywhere, 4x4 subdomains, 2 levels, corners.
    2. 3D elasticity 48^3 hex, E=1, nu=0.3, b=(0,0,-1), x=0 clamped, 4^3 subdomains of 12^3;
       2 levels, or 3 levels with 2x2x2 groups (``levels=3``, the default here).
    3. 3D elasticity 96^3, 12^3 subdomains of 8^3, E = 10^(3U); 3 levels (4x4x4 groups, the
       default here), 4 levels (2x2x2 groups twice: 1728 / 216 / 27) or 2 levels.
    4. 3D elasticity 80^3 cut by seeded random planes into 8^3 uneven boxes, 3 levels (2x2x2).
    5. 3D elasticity 64^3, 8^3 subdomains of 8^3, 3 levels (2x2x2), E = exp(theta), theta~N(0, 0.5^2).
    6. 3D elasticity 40^3, 2^3 subdomains of 20^3 (27,783 DOFs each), 2 levels, E = 10^(2U)
       (``large_subdomains``, its own seed 3).
    """
    name = CONFIG_NAMES[k]
    if k == 1:
        return box_workload(name, "poisson", (32, 32), [uniform_cuts(32, 4)] * 2,
                            dirichlet="all", constraints="c", seed=seed)
    if k == 2:
        lv = 3 if levels is None else levels
        groups = [(2, 2, 2)] if lv == 3 else []
        if lv not in (2, 3):
            raise ValueError("config 2 runs with 2 or 3 levels")
        return box_workload(name.replace("_64sub", f"_64sub_L{lv}"), "elasticity", (48,) * 3,
                            [uniform_cuts(48, 4)] * 3, groups=groups, seed=seed)
    if k == 3:
        n = 96 ** 3
        rng = np.random.default_rng(seed)
        young = 10.0 ** (3.0 * rng.random(n))
        lv = 3 if levels is None else levels
        if lv not in (2, 3, 4):
            raise ValueError("config 3 runs with 2, 3 or 4 levels")
        # 3 levels: 1728 / 27 / 1 (4x4x4 groups); 4 levels: 1728 / 216 / 27 / 1 (2x2x2 twice)
        groups = {2: [], 3: [(4, 4, 4)], 4: [(2, 2, 2), (2, 2, 2)]}[lv]
        return box_workload(f"{name}_L{lv}", "elasticity", (96,) * 3, [uniform_cuts(96, 12)] * 3,
                            groups=groups, young=young, seed=seed)
    if k == 4:
        cuts = random_cuts(seed)
        return box_workload(name, "elasticity", (80,) * 3, cuts, groups=[(2, 2, 2)], seed=seed)
    if k == 5:
        n = 64 ** 3
        rng = np.random.default_rng(seed)
        theta = rng.normal(0.0, 0.5, n)
        return box_workload(name, "elasticity", (64,) * 3, [uniform_cuts(64, 8)] * 3,
                            groups=[(2, 2, 2)], young=np.exp(theta), seed=seed)
    if k == 6:
        return large_subdomains()
    raise KeyError(k)
