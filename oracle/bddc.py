"""Oracle: the multilevel BDDC preconditioner (test infrastructure only).

Set-up follows Algorithm 1 of the paper: level 1 is built from the FE mesh;
for every further level the subdomains of the previous level become
'elements' with matrices K_Ci and their constrained globs become 'nodes'
(the pseudo-mesh), grouped into the next level's subdomains; the top coarse
matrix is factorized directly (dense Cholesky).

The apply follows Algorithm 2 and section 2:
  r_i = E_i^T r^                                (distribute the residual)
  [K_i C_i^T; C_i 0][z_i; lambda_i] = [r_i; 0]  (Eq. (2), subdomain correction)
  r_C = sum_i R_Ci^T Psi_i^T E_i^T r^            (coarse residual)
  K_C z_C = r_C  at the top level, otherwise one BDDC step of the next level
  z^ = sum_i E_i (Psi_i R_Ci z_C + z_i)          (combine and average)
On levels l > 1 the input is a whole vector of the previous level's coarse
space; it is first corrected in the subdomain interiors and the result is
post-corrected (the interior pre-/post-correction of section 2).  The paper
names these steps without writing them out; the reading used is block
elimination of the interiors:
  u_I = K_II^{-1} r_I,  r^ = r_G - sum K_GI u_I,  z^ = BDDC(r^),
  z_I = u_I - K_II^{-1} K_IG z^.
"""

from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from .dd import Level, dense_cholesky_solve, level_one_blocks
from .fem import dof_numbering, reference_element_matrix


class MultilevelBDDC:
    """Explicit multilevel BDDC for a workload.

    ``constraints`` may give one constraint mode per level (see ``Level``);
    ``n_levels`` defaults to the workload's.
    """

    def __init__(self, w, n_levels: Optional[int] = None, constraints: Optional[Sequence[str]] = None,
                 weights: str = "stiffness", structure_only: bool = False, level1: Optional[Level] = None):
        """``level1``: a level 1 already built for the same mesh, partition,
        moduli, level-1 constraints and weights (it depends on nothing else),
        reused instead of built again."""
        L = w.n_levels if n_levels is None else n_levels
        if L < 2 or L - 2 > len(w.sub_to_parent):
            raise ValueError("not enough level groupings for the requested number of levels")
        if constraints is None:
            constraints = [w.constraints] * (L - 1)
        self.n_levels = L
        Ke0 = reference_element_matrix(w)
        self.Ke0 = Ke0
        node_to_free, n_free = dof_numbering(w)
        self.node_to_free, self.n_free = node_to_free, n_free
        if level1 is None:
            blocks = level_one_blocks(w, Ke0, node_to_free)
            level1 = Level(w.dim, w.ndof, n_free // w.ndof, blocks, constraints[0], weights, structure_only)
            del blocks  # the element matrices (E_e K_e^0 per element) are no longer needed
        levels: List[Level] = [level1]
        for l in range(2, L):
            prev = levels[-1]
            parent = np.asarray(w.sub_to_parent[l - 2])
            el = prev.next_level_blocks()
            grouped = [[el[i] for i in np.nonzero(parent == p)[0]] for p in range(int(parent.max()) + 1)]
            levels.append(Level(w.dim, w.ndof, prev.n_coarse_nodes, grouped, constraints[l - 1], weights,
                                structure_only))
        self.levels = levels
        if not structure_only:
            self.top_solve = dense_cholesky_solve(levels[-1].KC)

    # ----------------------------------------------------------------- apply
    def apply(self, r_hat: np.ndarray) -> np.ndarray:
        """z^ = M_BDDC r^ on the level-1 interface."""
        return self._interface(0, np.asarray(r_hat, dtype=np.float64))

    def _interface(self, l: int, r_hat: np.ndarray) -> np.ndarray:
        lev = self.levels[l]
        r_C = np.zeros(lev.n_coarse)
        z_loc, r_loc = [], []
        for i in range(lev.n_sub):
            n_i = len(lev.sub_dofs[i])
            r_i = np.zeros(n_i)
            r_i[lev.loc_G[i]] = lev.D[i] * r_hat[lev.R[i]]           # E_i^T r^
            nc = lev.C[i].shape[0]
            sol = lev.saddle_lu[i].solve(np.concatenate([r_i, np.zeros(nc)]))   # Eq. (2)
            z_loc.append(sol[:n_i])
            np.add.at(r_C, lev.RC[i], lev.Psi[i].T @ r_i)            # R_Ci^T Psi_i^T E_i^T r^
        if l == len(self.levels) - 1:
            z_C = self.top_solve(r_C)
        else:
            z_C = self._full(l + 1, r_C)
        z_hat = np.zeros(lev.n_iface)
        for i in range(lev.n_sub):
            y = lev.Psi[i] @ z_C[lev.RC[i]] + z_loc[i]
            np.add.at(z_hat, lev.R[i], lev.D[i] * y[lev.loc_G[i]])    # E_i (...)
        return z_hat

    def _full(self, l: int, r: np.ndarray) -> np.ndarray:
        """One BDDC step on a whole level-l vector with interior pre/post-correction."""
        lev = self.levels[l]
        r_hat = r[lev.iface_dofs].copy()
        u = np.zeros(lev.n_dofs)
        for i in range(lev.n_sub):
            if lev.KII_lu[i] is None:
                continue
            dI = lev.sub_dofs[i][lev.loc_I[i]]
            uI = lev.KII_lu[i].solve(r[dI])
            u[dI] = uI
            np.add.at(r_hat, lev.R[i], -(lev.KIG[i].T @ uI))
        z_hat = self._interface(l, r_hat)
        z = np.zeros(lev.n_dofs)
        z[lev.iface_dofs] = z_hat
        for i in range(lev.n_sub):
            if lev.KII_lu[i] is None:
                continue
            dI = lev.sub_dofs[i][lev.loc_I[i]]
            z[dI] = u[dI] - lev.KII_lu[i].solve(lev.KIG[i] @ z_hat[lev.R[i]])
        return z

    # ------------------------------------------------------------ operators
    @property
    def level1(self) -> Level:
        return self.levels[0]

    def schur_apply(self, v: np.ndarray) -> np.ndarray:
        return self.level1.schur_apply(v)

    def condense(self, f: np.ndarray) -> np.ndarray:
        return self.level1.condense(f)

    def recover(self, f: np.ndarray, u_hat: np.ndarray) -> np.ndarray:
        return self.level1.recover(f, u_hat)

    def coarse_sizes(self) -> List[int]:
        return [lev.n_coarse for lev in self.levels]
