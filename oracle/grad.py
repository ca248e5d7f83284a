"""Oracle: compliance gradient (test infrastructure only).

For J = f^T u with K(theta) u = f and element moduli E_e = exp(theta_e), the
adjoint equation K lambda = dJ/du = f gives lambda, and
dJ/dtheta_e = -lambda_e^T (dK_e/dtheta_e) u_e = -E_e lambda_e^T K_e^0 u_e.
"""

from __future__ import annotations

import numpy as np

from .fem import dof_numbering, element_dofs, reference_element_matrix


def element_energy(w, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out_e = E_e a_e^T K_e^0 b_e for free-DOF vectors a, b (eliminated DOFs are zero)."""
    node_to_free, _ = dof_numbering(w)
    ed = element_dofs(w, node_to_free)
    Ke0 = reference_element_matrix(w)
    ae = np.where(ed >= 0, a[np.maximum(ed, 0)], 0.0)
    be = np.where(ed >= 0, b[np.maximum(ed, 0)], 0.0)
    return w.young * np.einsum("ei,ij,ej->e", ae, Ke0, be)


def compliance_gradient(w, u: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """dJ/dtheta_e for J = f^T u (lam solves the adjoint system K lam = f)."""
    return -element_energy(w, lam, u)
