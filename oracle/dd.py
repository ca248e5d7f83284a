"""Oracle: one level of the BDDC hierarchy (test infrastructure only).

Follows section 2 and the body of Algorithm 1 of the paper:

* local subdomain matrices K_i by sub-assembly of element matrices;
* the interface = level nodes shared by two or more subdomains;
* interface classification into faces / edges / vertices (globs = classes of
  interface nodes with the same set of subdomains, each split into the parts
  that elements connect) and corner selection;
* the constraint matrix C_i (one row per constraint: corner values, and
  arithmetic averages over edges and faces, per component);
* the weights E_i that distribute the interface residual;
* the coarse basis Psi_i and Lambda_i from the saddle-point problem of
  Eq. (1), the local coarse matrices K_Ci = -Lambda_i and their assembly K_C.

Readings where the paper is silent (kept identical in the GPU library):

* a glob is a connected part of a class of interface nodes with the same
  subdomain set, two nodes of a class being connected when one element holds
  both (on box partitions every class is connected; on general partitions two
  subdomains can touch in separate patches, each of which gets its own
  averages);
* corner selection: a glob shared by three or more subdomains that consists
  of a single node is a corner; in 3D a glob of two subdomains is a face and
  one of three or more subdomains with several nodes is an edge; in 2D a glob
  of two subdomains is an edge (no further corners are selected on general
  partitions: the face-based algorithm the paper uses is not described
  there);
* Dirichlet nodes are removed before the interface is formed, so a glob that
  touches the Dirichlet boundary keeps only its free nodes;
* averages use equal weights 1/m over the m nodes of a glob, one row per
  component; on higher levels the same holds over pseudo-nodes;
* weights are the diagonal-stiffness ratios D_i(k) = K_i(k,k) / sum_j K_j(k,k)
  (or the multiplicity 1/#subdomains as a variant);
* globs are ordered by their smallest node index; coarse DOFs are numbered
  glob by glob, component innermost.

Factorizations are sparse LU (scipy.sparse.linalg.splu) of the full matrices;
nothing of the GPU library's Schur-complement algebra is reused here.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Sequence, Tuple

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

CORNER, EDGE, FACE = 0, 1, 2
KIND_NAMES = {CORNER: "corner", EDGE: "edge", FACE: "face"}


@dataclass
class Glob:
    nodes: np.ndarray          # level node ids, sorted
    subs: Tuple[int, ...]      # sorted subdomain ids sharing the glob
    kind: int                  # CORNER / EDGE / FACE
    constrained: bool = False  # carries coarse DOFs
    coarse_node: int = -1      # pseudo-node id on the next level


def classify(n_subs: int, n_nodes: int, dim: int) -> int:
    """Glob type from the number of subdomains sharing it and its node count."""
    if n_subs >= 3 and n_nodes == 1:
        return CORNER
    if n_subs == 2:
        return FACE if dim == 3 else EDGE
    return EDGE


class Level:
    """One level: subdomains made of elements with given matrices.

    Parameters
    ----------
    dim, ndof : geometric dimension and DOFs per node.
    n_nodes   : number of (free) nodes of this level; DOF = node * ndof + c.
    blocks    : per subdomain, a list of element blocks ``(edofs, mats)`` with
                ``edofs`` int [m, nloc] (level DOF or -1 for an eliminated DOF)
                and ``mats`` float [m, nloc, nloc].
    constraints : "c" corners only, "cef" corners + edge and face averages,
                "primal" every interface node is its own corner.
    weights   : "stiffness" or "multiplicity".
    """

    def __init__(self, dim: int, ndof: int, n_nodes: int, blocks: Sequence[List[Tuple[np.ndarray, np.ndarray]]],
                 constraints: str = "cef", weights: str = "stiffness", structure_only: bool = False):
        self.dim, self.ndof, self.n_nodes = dim, ndof, n_nodes
        self.n_dofs = n_nodes * ndof
        self.n_sub = len(blocks)
        self.constraints, self.weights = constraints, weights
        nd = ndof

        # --- subdomain matrices by sub-assembly (K_i, section 2)
        self.sub_dofs: List[np.ndarray] = []
        self.K: List[sp.csr_matrix] = []
        for blk in blocks:
            rows, cols, vals = [], [], []
            for edofs, mats in blk:
                nloc = edofs.shape[1]
                r = np.repeat(edofs, nloc, axis=1).ravel()
                c = np.tile(edofs, (1, nloc)).ravel()
                v = np.asarray(mats).reshape(len(edofs), -1).ravel()
                keep = (r >= 0) & (c >= 0)
                rows.append(r[keep]); cols.append(c[keep]); vals.append(v[keep])
            rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
            dofs = np.unique(rows)
            loc = np.searchsorted(dofs, rows), np.searchsorted(dofs, cols)
            Ki = sp.coo_matrix((vals, loc), shape=(len(dofs), len(dofs))).tocsr()
            self.sub_dofs.append(dofs)
            self.K.append(Ki)

        # --- nodes of each subdomain and their subdomain sets
        self.sub_nodes = [np.unique(d // nd) for d in self.sub_dofs]
        node_subs: Dict[int, List[int]] = {}
        for i, nodes in enumerate(self.sub_nodes):
            for n in nodes.tolist():
                node_subs.setdefault(n, []).append(i)
        self.node_subs = node_subs
        iface_nodes = sorted(n for n, s in node_subs.items() if len(s) >= 2)
        self.iface_nodes = np.array(iface_nodes, dtype=np.int64)

        # --- globs (interface classification) and corners
        groups: Dict[Tuple[int, ...], List[int]] = {}
        for n in iface_nodes:
            groups.setdefault(tuple(node_subs[n]), []).append(n)
        globs = []
        if constraints == "primal":
            for n in iface_nodes:
                globs.append(Glob(np.array([n]), tuple(node_subs[n]), CORNER))
        else:
            part = self._connected_parts(blocks, groups)
            for subs, nodes in groups.items():
                nodes = np.array(sorted(nodes))
                for lab in np.unique(part[nodes]):
                    g_nodes = nodes[part[nodes] == lab]
                    globs.append(Glob(g_nodes, subs, classify(len(subs), len(g_nodes), dim)))
        globs.sort(key=lambda g: int(g.nodes[0]))
        n_coarse_nodes = 0
        for g in globs:
            g.constrained = g.kind == CORNER or constraints in ("cef",)
            if g.constrained:
                g.coarse_node = n_coarse_nodes
                n_coarse_nodes += 1
        self.globs = globs
        self.n_coarse_nodes = n_coarse_nodes
        self.n_coarse = n_coarse_nodes * nd

        # --- global interface DOF numbering (increasing level DOF)
        iface_dofs = (self.iface_nodes[:, None] * nd + np.arange(nd)[None, :]).ravel()
        self.iface_dofs = iface_dofs
        self.n_iface = len(iface_dofs)
        dof_to_iface = -np.ones(self.n_dofs, dtype=np.int64)
        dof_to_iface[iface_dofs] = np.arange(self.n_iface)
        self.dof_to_iface = dof_to_iface
        is_iface_dof = dof_to_iface >= 0

        # --- per-subdomain interior / interface split, C_i, R_Ci
        self.loc_I, self.loc_G, self.R = [], [], []   # local index lists, R_i: local iface -> global iface
        self.C: List[sp.csr_matrix] = []
        self.RC: List[np.ndarray] = []                # R_Ci: local coarse -> global coarse
        for i in range(self.n_sub):
            dofs = self.sub_dofs[i]
            isg = is_iface_dof[dofs]
            self.loc_I.append(np.nonzero(~isg)[0])
            self.loc_G.append(np.nonzero(isg)[0])
            self.R.append(dof_to_iface[dofs[isg]])
            crow, ccol, cval, rc = [], [], [], []
            row = 0
            for g in globs:
                if not g.constrained or i not in g.subs:
                    continue
                m = len(g.nodes)
                for c in range(nd):
                    gd = g.nodes * nd + c
                    ld = np.searchsorted(dofs, gd)
                    crow.extend([row] * m); ccol.extend(ld.tolist()); cval.extend([1.0 / m] * m)
                    rc.append(g.coarse_node * nd + c)
                    row += 1
            self.C.append(sp.coo_matrix((cval, (crow, ccol)), shape=(row, len(dofs))).tocsr())
            self.RC.append(np.array(rc, dtype=np.int64))

        # --- weights D_i on the local interface DOFs; E_i^T r = D_i (R_i r)
        # (index structure only: the matrices of levels >= 2 are not formed, so
        # the multiplicity weights stand in for the stiffness ratios)
        if weights == "stiffness" and not structure_only:
            diag_sum = np.zeros(self.n_iface)
            diags = []
            for i in range(self.n_sub):
                d = self.K[i].diagonal()[self.loc_G[i]]
                diags.append(d)
                np.add.at(diag_sum, self.R[i], d)
            self.D = [diags[i] / diag_sum[self.R[i]] for i in range(self.n_sub)]
        elif weights in ("multiplicity", "stiffness"):
            mult = np.zeros(self.n_iface)
            for i in range(self.n_sub):
                np.add.at(mult, self.R[i], 1.0)
            self.D = [1.0 / mult[self.R[i]] for i in range(self.n_sub)]
        else:
            raise ValueError(weights)

        if structure_only:
            # index structure only (interface, globs, coarse numbering); no factorizations
            self.KC_loc = [np.zeros((len(rc), len(rc))) for rc in self.RC]
            return

        # --- interior factorizations (Algorithm 1: interior correction / Dirichlet problems)
        self.KII_lu, self.KIG, self.KGG = [], [], []
        for i in range(self.n_sub):
            Ki = self.K[i]
            I, G = self.loc_I[i], self.loc_G[i]
            KII = Ki[I][:, I].tocsc()
            # symmetric pattern: minimum degree on A^T + A keeps the fill lowest
            self.KII_lu.append(spla.splu(KII, permc_spec="MMD_AT_PLUS_A") if len(I) else None)
            self.KIG.append(Ki[I][:, G].tocsr())
            self.KGG.append(Ki[G][:, G].tocsr())

        # --- saddle-point factorization and coarse basis, Eq. (1)
        self.saddle_lu, self.Psi, self.Lam, self.KC_loc = [], [], [], []
        for i in range(self.n_sub):
            Ki, Ci = self.K[i], self.C[i]
            nc = Ci.shape[0]
            A = sp.bmat([[Ki, Ci.T], [Ci, None]], format="csc")
            # the local node order is already banded; keeping it (with the
            # constraint rows last) gives less fill than a column ordering
            # here, and the factors of every subdomain are kept for the applies
            lu = spla.splu(A, permc_spec="NATURAL")
            rhs = np.zeros((Ki.shape[0] + nc, nc))
            rhs[Ki.shape[0]:, :] = np.eye(nc)
            sol = lu.solve(rhs) if nc else np.zeros((Ki.shape[0], 0))
            self.saddle_lu.append(lu)
            self.Psi.append(np.ascontiguousarray(sol[:Ki.shape[0], :]))
            self.Lam.append(np.ascontiguousarray(sol[Ki.shape[0]:, :]))
            self.KC_loc.append(-self.Lam[-1])

        # --- global coarse matrix K_C = sum R_Ci^T K_Ci R_Ci
        KC = np.zeros((self.n_coarse, self.n_coarse))
        for i in range(self.n_sub):
            rc = self.RC[i]
            KC[np.ix_(rc, rc)] += self.KC_loc[i]
        self.KC = KC

    # ------------------------------------------------------------------ Schur
    def _connected_parts(self, blocks, groups) -> np.ndarray:
        """Label of the connected part of every node: nodes of one class of
        `groups` are joined when an element holds both."""
        nd = self.ndof
        cls = -np.ones(self.n_nodes, dtype=np.int64)
        for c, nodes in enumerate(groups.values()):
            cls[np.asarray(nodes, dtype=np.int64)] = c
        rows, cols = [], []
        for blk in blocks:
            for edofs, _ in blk:
                e = np.asarray(edofs)
                nn = e.shape[1] // nd
                # node of each element slot (its DOFs are node * nd + c; -1 where eliminated)
                en = np.stack([e[:, k * nd:(k + 1) * nd].max(axis=1) for k in range(nn)], axis=1)
                en = np.where(en >= 0, en // nd, -1)
                for p in range(nn):
                    for q in range(p + 1, nn):
                        a, b = en[:, p], en[:, q]
                        ok = (a >= 0) & (b >= 0)
                        a, b = a[ok], b[ok]
                        same = (cls[a] >= 0) & (cls[a] == cls[b])
                        rows.append(a[same]); cols.append(b[same])
        rows = np.concatenate(rows) if rows else np.zeros(0, dtype=np.int64)
        cols = np.concatenate(cols) if cols else np.zeros(0, dtype=np.int64)
        A = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(self.n_nodes, self.n_nodes))
        from scipy.sparse.csgraph import connected_components
        return connected_components(A, directed=False)[1]

    def schur_local(self, i: int, v_loc: np.ndarray) -> np.ndarray:
        """S_i v = K_GG v - K_GI K_II^{-1} K_IG v (a discrete Dirichlet problem)."""
        y = self.KGG[i] @ v_loc
        if self.KII_lu[i] is not None:
            y -= self.KIG[i].T @ self.KII_lu[i].solve(self.KIG[i] @ v_loc)
        return y

    def schur_apply(self, v: np.ndarray) -> np.ndarray:
        """S^ v = sum_i R_i^T S_i R_i v, without forming S^ (section 2)."""
        out = np.zeros(self.n_iface)
        for i in range(self.n_sub):
            np.add.at(out, self.R[i], self.schur_local(i, v[self.R[i]]))
        return out

    def schur_dense(self, i: int) -> np.ndarray:
        KIG = self.KIG[i].toarray()
        if self.KII_lu[i] is None:
            return self.KGG[i].toarray()
        return self.KGG[i].toarray() - KIG.T @ self.KII_lu[i].solve(KIG)

    def condense(self, f: np.ndarray) -> np.ndarray:
        """g^ = f_Gamma - sum_i R_i^T K_GI K_II^{-1} f_I (condensed right-hand side)."""
        g = f[self.iface_dofs].copy()
        for i in range(self.n_sub):
            if self.KII_lu[i] is None:
                continue
            fI = f[self.sub_dofs[i][self.loc_I[i]]]
            np.add.at(g, self.R[i], -(self.KIG[i].T @ self.KII_lu[i].solve(fI)))
        return g

    def recover(self, f: np.ndarray, u_hat: np.ndarray) -> np.ndarray:
        """Full solution from the interface part: u_I = K_II^{-1}(f_I - K_IG u_G)."""
        u = np.zeros(self.n_dofs)
        u[self.iface_dofs] = u_hat
        for i in range(self.n_sub):
            if self.KII_lu[i] is None:
                continue
            dI = self.sub_dofs[i][self.loc_I[i]]
            u[dI] = self.KII_lu[i].solve(f[dI] - self.KIG[i] @ u_hat[self.R[i]])
        return u

    # --------------------------------------------------------------- counts
    def glob_counts(self) -> Dict[str, int]:
        out = {"corner": 0, "edge": 0, "face": 0}
        for g in self.globs:
            out[KIND_NAMES[g.kind]] += 1
        return out

    def next_level_blocks(self):
        """Pseudo-mesh for the next level (Algorithm 1): subdomains become
        elements with matrices K_Ci; constrained globs become nodes with ndof
        DOFs each.  Returns one single-element block per subdomain."""
        return [(self.RC[i][None, :], self.KC_loc[i][None, :, :]) for i in range(self.n_sub)]


def level_one_blocks(w, Ke0: np.ndarray, node_to_free: np.ndarray) -> List[List[Tuple[np.ndarray, np.ndarray]]]:
    """Element blocks of every level-1 subdomain with E_e K_e^0 matrices."""
    from .fem import element_dofs
    edofs = element_dofs(w, node_to_free)
    blocks = []
    order = np.argsort(w.elem_to_sub, kind="stable")
    bounds = np.searchsorted(w.elem_to_sub[order], np.arange(w.n_subdomains + 1))
    for i in range(w.n_subdomains):
        els = order[bounds[i]:bounds[i + 1]]
        mats = w.young[els][:, None, None] * Ke0[None, :, :]
        blocks.append([(edofs[els], mats)])
    return blocks


def dense_cholesky_solve(A: np.ndarray):
    """Factor once, return a solver (top-level coarse problem, Algorithm 1)."""
    c = sla.cho_factor(A, lower=True)
    return lambda b: sla.cho_solve(c, b)
