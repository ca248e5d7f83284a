"""Oracle: direct solves used as ground truth (test infrastructure only)."""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fem import assemble_global


def direct_solve(w):
    """Solution of the global FE system K u = f on the free DOFs (sparse LU)."""
    K, f = assemble_global(w)
    u = spla.splu(K.tocsc()).solve(f)
    return u, K, f


def solve_bddc(w, bddc=None, tol: float = 1e-8, max_iter: int = 1000, **kw):
    """Condense, run BDDC-PCG on the interface, recover the interior."""
    from .bddc import MultilevelBDDC
    from .krylov import pcg
    if bddc is None:
        bddc = MultilevelBDDC(w, **kw)
    _, f = assemble_global(w)
    g = bddc.condense(f)
    res = pcg(bddc.schur_apply, g, bddc.apply, tol=tol, max_iter=max_iter)
    u = bddc.recover(f, res.x)
    return u, res, bddc, f
