"""Oracle FE discretisation of the model problems (test infrastructure only).

The paper discretises its problems with tetrahedra and Taylor-Hood elements
(section 4); the synthetic workloads here use the structured Q1 / trilinear
hexahedral analogues.  Everything is FP64 and written for clarity:

* 2D Poisson: bilinear Q1 element on a square, stiffness in closed form.
* 3D linear elasticity: trilinear hexahedron, isotropic Hooke law, 2x2x2
  Gauss quadrature.  The matrix of an element with modulus E is E times the
  matrix of the unit-modulus element.
* Consistent load of a constant source/body force.
* Homogeneous Dirichlet nodes are eliminated.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def q1_laplace_element() -> np.ndarray:
    """Stiffness of -Laplace on one square bilinear element (any size in 2D):
    integral of grad N_a . grad N_b, nodes counter-clockwise from (0,0)."""
    return np.array([[4.0, -1.0, -2.0, -1.0],
                     [-1.0, 4.0, -1.0, -2.0],
                     [-2.0, -1.0, 4.0, -1.0],
                     [-1.0, -2.0, -1.0, 4.0]]) / 6.0


# reference coordinates of the hexahedron's nodes, in the workloads' local order
HEX_NODES = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                      [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)


def isotropic_d(E: float, nu: float) -> np.ndarray:
    """Hooke matrix in Voigt order (xx, yy, zz, yz, xz, xy), engineering shears."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def hex8_shape_gradients(xi: np.ndarray, h: float) -> np.ndarray:
    """Physical gradients dN_a/dx (8 x 3) of the trilinear shape functions of a
    cube of side h at reference point xi; the Jacobian is (h/2) I."""
    g = np.zeros((8, 3))
    for a in range(8):
        s = HEX_NODES[a]
        f = 1.0 + s * xi
        g[a, 0] = s[0] * f[1] * f[2] / 8.0
        g[a, 1] = f[0] * s[1] * f[2] / 8.0
        g[a, 2] = f[0] * f[1] * s[2] / 8.0
    return g * (2.0 / h)


def hex8_strain_matrix(dN: np.ndarray) -> np.ndarray:
    """B (6 x 24) mapping element DOFs (node-major, 3 components) to Voigt strain."""
    B = np.zeros((6, 24))
    for a in range(8):
        dx, dy, dz = dN[a]
        c = 3 * a
        B[0, c + 0] = dx
        B[1, c + 1] = dy
        B[2, c + 2] = dz
        B[3, c + 1] = dz; B[3, c + 2] = dy
        B[4, c + 0] = dz; B[4, c + 2] = dx
        B[5, c + 0] = dy; B[5, c + 1] = dx
    return B


def hex8_elasticity_element(E: float, nu: float, h: float) -> np.ndarray:
    """Stiffness of a cube element of side h, 2x2x2 Gauss rule."""
    D = isotropic_d(E, nu)
    g = 1.0 / np.sqrt(3.0)
    detJ = (h / 2.0) ** 3
    K = np.zeros((24, 24))
    for p in (-g, g):
        for q in (-g, g):
            for r in (-g, g):
                B = hex8_strain_matrix(hex8_shape_gradients(np.array([p, q, r]), h))
                K += B.T @ D @ B * detJ
    return K


def reference_element_matrix(w) -> np.ndarray:
    """Unit-modulus element matrix K_e^0 of a workload."""
    if w.physics == "poisson":
        return q1_laplace_element()
    return hex8_elasticity_element(1.0, w.poisson_ratio, w.h)


def element_load(w) -> np.ndarray:
    """Consistent load of a constant source / body force on one element:
    each node receives (element volume / number of nodes) times the force,
    since every bilinear/trilinear shape function integrates to that share."""
    nn = 2 ** w.dim
    vol = w.h ** w.dim
    share = vol / nn
    return np.tile(np.asarray(w.body_force, dtype=np.float64) * share, nn)


def dof_numbering(w):
    """Free-DOF numbering: free nodes in increasing node order, components
    innermost.  Returns (node -> free-node index or -1, number of free DOFs)."""
    free = ~w.dirichlet_nodes
    node_to_free = -np.ones(w.n_nodes, dtype=np.int64)
    node_to_free[free] = np.arange(int(free.sum()))
    return node_to_free, int(free.sum()) * w.ndof


def element_dofs(w, node_to_free) -> np.ndarray:
    """Free-DOF index (or -1) of every element DOF, node-major."""
    fn = node_to_free[w.elem_nodes]                      # [n_elems, nn]
    nd = w.ndof
    dofs = fn[:, :, None] * nd + np.arange(nd)[None, None, :]
    dofs[fn < 0] = -1
    return dofs.reshape(len(w.elem_nodes), -1)


def assemble_global(w):
    """Global stiffness on free DOFs (CSR) and the load vector."""
    node_to_free, n = dof_numbering(w)
    edofs = element_dofs(w, node_to_free)
    Ke0 = reference_element_matrix(w)
    nloc = edofs.shape[1]
    rows = np.repeat(edofs, nloc, axis=1)
    cols = np.tile(edofs, (1, nloc))
    vals = w.young[:, None] * Ke0.ravel()[None, :]
    keep = (rows >= 0) & (cols >= 0)
    K = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    return K, load_vector(w)


def load_vector(w) -> np.ndarray:
    """Load vector on the free DOFs: every element's consistent load added
    at its free DOFs (the right-hand side of assemble_global, without the
    matrix)."""
    node_to_free, n = dof_numbering(w)
    edofs = element_dofs(w, node_to_free)
    fe = element_load(w)
    f = np.zeros(n)
    fv = np.broadcast_to(fe, edofs.shape)
    np.add.at(f, edofs[edofs >= 0], fv[edofs >= 0])
    return f


def total_load(w) -> np.ndarray:
    """Sum of all nodal loads per component before Dirichlet elimination."""
    fe = element_load(w).reshape(2 ** w.dim, w.ndof)
    return fe.sum(axis=0) * w.n_elems
