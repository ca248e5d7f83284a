"""Python front-end of the MI355X multilevel BDDC library.

`Problem` turns a structured-mesh problem description into the C ABI's mesh
and partition arrays (element matrices and loads come from the library's own
host routines).  `Solver` owns a library handle; its methods pass torch
device buffers and the current HIP stream to the library and do nothing
else.  `BDDCSolve` is the autograd wrapper: forward solves K(theta) u = f,
backward reuses the same BDDC-PCG for the adjoint system and forms the
element sensitivities in a library kernel.
"""

from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

TUNE_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.txt")

_CONSTRAINTS = {
    "c": L.MLBDDC_CORNERS,
    "ce": L.MLBDDC_CORNERS | L.MLBDDC_EDGES,
    "cf": L.MLBDDC_CORNERS | L.MLBDDC_FACES,
    "cef": L.MLBDDC_CORNERS | L.MLBDDC_EDGES | L.MLBDDC_FACES,
    "primal": L.MLBDDC_ALL_PRIMAL,
}


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def element_matrix(kind: int, h: float, nu: float = 0.3) -> np.ndarray:
    n = 4 if kind == L.MLBDDC_POISSON_Q1 else 24
    out = np.zeros((n, n))
    L.check(L.load().mlbddc_element_matrix(kind, h, nu, _ptr(out, C.c_double)))
    return out


def element_load(kind: int, h: float, force: Sequence[float]) -> np.ndarray:
    n = 4 if kind == L.MLBDDC_POISSON_Q1 else 24
    f = np.ascontiguousarray(force, dtype=np.float64)
    out = np.zeros(n)
    L.check(L.load().mlbddc_element_load(kind, h, _ptr(f, C.c_double), _ptr(out, C.c_double)))
    return out


def _torch_allocator(device: torch.device, stream) -> "L.Allocator":
    """The library's device allocator: torch's caching allocator on the
    handle's stream (torch owns every device block the library uses)."""

    def alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
        except Exception:  # out of memory: the library reports E_NOMEM
            return None

    def free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a = L.Allocator(L.ALLOC_FN(alloc), L.FREE_FN(free), None)
    a._keep = (alloc, free)
    return a


# Handles still alive at interpreter exit are destroyed while torch is still usable.
_LIVE: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _destroy_live():
    for s in list(_LIVE):
        try:
            s.destroy()
        except Exception:
            pass


class Problem:
    """Mesh + partition arrays of a structured problem in the C-ABI layout."""

    def __init__(self, w, constraints: Optional[str] = None, n_levels: Optional[int] = None):
        self.kind = L.MLBDDC_POISSON_Q1 if w.physics == "poisson" else L.MLBDDC_ELASTICITY_HEX8
        self.dim = int(w.dim)
        self.ndof = 1 if w.physics == "poisson" else self.dim
        self.h = float(w.h)
        self.Ke0 = element_matrix(self.kind, self.h, float(w.poisson_ratio))
        self.elem_nodes = np.ascontiguousarray(w.elem_nodes, dtype=np.int32)
        self.n_elems = int(self.elem_nodes.shape[0])
        self.nodes_per_elem = int(self.elem_nodes.shape[1])
        self.n_nodes = int(np.prod([n + 1 for n in w.n_el]))
        self.scale = np.ascontiguousarray(w.young, dtype=np.float64)
        self.dirichlet = np.ascontiguousarray(w.dirichlet_nodes, dtype=np.uint8)
        self.elem_to_sub = np.ascontiguousarray(w.elem_to_sub, dtype=np.int32)
        self.n_levels = int(w.n_levels if n_levels is None else n_levels)
        self.parents = [np.ascontiguousarray(p, dtype=np.int32) for p in w.sub_to_parent][: max(self.n_levels - 2, 0)]
        if len(self.parents) < self.n_levels - 2:
            raise ValueError("not enough level groupings for the requested number of levels")
        self.constraints = _CONSTRAINTS[constraints or w.constraints]
        self.body_force = np.asarray(w.body_force, dtype=np.float64)
        free = self.dirichlet == 0
        self.node_to_free = np.full(self.n_nodes, -1, dtype=np.int64)
        self.node_to_free[free] = np.arange(int(free.sum()))
        self.n_dofs = int(free.sum()) * self.ndof

    def structs(self):
        """Build the ctypes mesh / partition structs (keep the returned tuple alive)."""
        m = L.Mesh(self.dim, self.ndof, self.n_nodes, self.n_elems, self.nodes_per_elem,
                   _ptr(self.elem_nodes, C.c_int32), _ptr(self.Ke0, C.c_double), _ptr(self.scale, C.c_double),
                   _ptr(self.dirichlet, C.c_uint8))
        parr = (C.POINTER(C.c_int32) * max(len(self.parents), 1))(*[_ptr(p, C.c_int32) for p in self.parents])
        p = L.Partition(self.n_levels, _ptr(self.elem_to_sub, C.c_int32), parr, self.constraints)
        return m, p, parr

    def load_vector(self) -> np.ndarray:
        """Consistent load of the constant source / body force on the free DOFs
        (assembled by the library's host routine)."""
        fe = element_load(self.kind, self.h, self.body_force)
        f = np.zeros(self.n_dofs)
        m, p, keep = self.structs()
        L.check(L.load().mlbddc_assemble_load(C.byref(m), _ptr(fe, C.c_double), _ptr(f, C.c_double), self.n_dofs))
        return f

    def counts(self):
        """Host-only plan summary per BDDC level: subdomains, interface, coarse, corners, edges, faces."""
        m, p, keep = self.structs()
        out = np.zeros((self.n_levels - 1, 6), dtype=np.int64)
        L.check(L.load().mlbddc_plan_counts(C.byref(m), C.byref(p), _ptr(out, C.c_int64)))
        return out


class Solver:
    """Handle of the HIP multilevel BDDC library on one device."""

    def __init__(self, precision: str = "fp64", rtol: float = 1e-8, max_iter: int = 1000, weights: str = "stiffness",
                 device: int = 0, panel_tiles: int = 0, use_graph: bool = False, panel_tiles_precond: int = 0,
                 tune_table: Optional[str] = TUNE_TABLE, lookahead: bool = False, side_stream: bool = True,
                 stage_cols: int = 0, mv_group_tiles: int = 0, mfma_f32: int = 0):
        lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the BDDC library needs a HIP device")
        self.lib = lib
        self.device = torch.device("cuda", device)
        opt = L.Options()
        lib.mlbddc_default_options(C.byref(opt))
        opt.precision = L.MLBDDC_MIXED if precision == "mixed" else L.MLBDDC_FP64
        opt.rtol = rtol
        opt.max_iter = max_iter
        opt.weights = L.MLBDDC_W_MULTIPLICITY if weights == "multiplicity" else L.MLBDDC_W_STIFFNESS
        opt.use_graph = 1 if use_graph else 0
        opt.panel_tiles = panel_tiles
        opt.panel_tiles_precond = panel_tiles_precond
        self._tune = tune_table.encode() if tune_table and os.path.exists(tune_table) else None
        opt.tune_table = self._tune
        opt.lookahead = 1 if lookahead else 0
        opt.side_stream = 1 if side_stream else 0
        opt.stage_cols = stage_cols
        opt.mv_group_tiles = mv_group_tiles
        opt.mfma_f32 = mfma_f32
        opt.device = device
        self.opt = opt
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        self._alloc = _torch_allocator(self.device, self.stream)
        h = C.c_void_p()
        L.check(lib.mlbddc_create(C.byref(h), C.byref(opt), C.byref(self._alloc), C.c_void_p(self.stream.cuda_stream)))
        self.h = h
        _LIVE.add(self)
        self.problem: Optional[Problem] = None

    def destroy(self):
        """Release the handle; its device blocks go back to torch's caching allocator."""
        if getattr(self, "h", None):
            self.lib.mlbddc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def _chk(self, st):
        L.check(st, self.h)

    # ----------------------------------------------------------------- setup
    def setup(self, prob: Problem):
        m, p, keep = prob.structs()
        self._chk(self.lib.mlbddc_setup(self.h, C.byref(m), C.byref(p)))
        self.problem = prob
        self.n_dofs = int(self.lib.mlbddc_num_dofs(self.h))
        self.n_iface = int(self.lib.mlbddc_interface_size(self.h))
        return self

    def update_coefficients(self, scale: torch.Tensor):
        s = scale.to(self.device, torch.float64).contiguous()
        self._chk(self.lib.mlbddc_update_coefficients(self.h, C.c_void_p(s.data_ptr())))

    def coarse_size(self, level: int) -> int:
        return int(self.lib.mlbddc_coarse_size(self.h, level))

    def num_subdomains(self, level: int) -> int:
        return int(self.lib.mlbddc_num_subdomains(self.h, level))

    # ------------------------------------------------------------- operators
    def _vec(self, v, n):
        t = torch.as_tensor(v, dtype=torch.float64, device=self.device).contiguous()
        if t.numel() != n:
            raise ValueError(f"expected {n} entries, got {t.numel()}")
        return t

    def apply(self, r) -> torch.Tensor:
        r = self._vec(r, self.n_iface)
        z = torch.empty_like(r)
        self._chk(self.lib.mlbddc_apply(self.h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr())))
        return z

    def apply_into(self, r: torch.Tensor, z: torch.Tensor):
        self._chk(self.lib.mlbddc_apply(self.h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr())))

    def apply_schur_into(self, x: torch.Tensor, y: torch.Tensor):
        self._chk(self.lib.mlbddc_apply_schur(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())))

    def apply_schur(self, x) -> torch.Tensor:
        x = self._vec(x, self.n_iface)
        y = torch.empty_like(x)
        self._chk(self.lib.mlbddc_apply_schur(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())))
        return y

    def condense(self, f) -> torch.Tensor:
        f = self._vec(f, self.n_dofs)
        g = torch.empty(self.n_iface, dtype=torch.float64, device=self.device)
        self._chk(self.lib.mlbddc_condense(self.h, C.c_void_p(f.data_ptr()), C.c_void_p(g.data_ptr())))
        return g

    def solve(self, f, u0=None, raise_on_error: bool = True):
        f = self._vec(f, self.n_dofs)
        u = torch.empty_like(f)
        st = L.Stats()
        u0p = C.c_void_p(self._vec(u0, self.n_dofs).data_ptr()) if u0 is not None else None
        status = self.lib.mlbddc_solve(self.h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), u0p, C.byref(st))
        if raise_on_error:
            self._chk(status)
        d = st.as_dict()
        d["status"] = L.STATUS.get(status, str(status))
        return u, d

    def element_energy(self, a, b) -> torch.Tensor:
        a = self._vec(a, self.n_dofs)
        b = self._vec(b, self.n_dofs)
        out = torch.empty(self.problem.n_elems, dtype=torch.float64, device=self.device)
        self._chk(self.lib.mlbddc_element_energy(self.h, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                                 C.c_void_p(out.data_ptr())))
        return out

    def interface_dofs(self) -> np.ndarray:
        """Free-DOF index of every level-1 interface entry (increasing)."""
        out = np.zeros(self.n_iface, dtype=np.int64)
        self._chk(self.lib.mlbddc_interface_dofs(self.h, _ptr(out, C.c_int64)))
        return out

    def subdomain_sizes(self, level: int) -> np.ndarray:
        """(interior DOFs, interface DOFs, constraints) of every level-`level` subdomain."""
        n = self.num_subdomains(level)
        out = np.zeros((n, 3), dtype=np.int64)
        self._chk(self.lib.mlbddc_subdomain_sizes(self.h, level, _ptr(out, C.c_int64)))
        return out

    def set_profiling(self, enable: bool = True):
        self._chk(self.lib.mlbddc_set_profiling(self.h, 1 if enable else 0))

    def profile(self) -> dict:
        p = L.Profile()
        self._chk(self.lib.mlbddc_get_profile(self.h, C.byref(p)))
        return p.as_dict()

    def coarse_matrix(self, level: int) -> np.ndarray:
        n = self.coarse_size(level)
        out = np.zeros((n, n))
        self._chk(self.lib.mlbddc_get_coarse_matrix(self.h, level, _ptr(out, C.c_double)))
        return out


class BDDCSolve(torch.autograd.Function):
    """u = K(theta)^{-1} f with K = sum_e exp(theta_e) K_e^0.

    The backward pass solves the adjoint system K lambda = dL/du with the same
    set-up and returns dL/dtheta_e = -lambda_e^T (dK_e/dtheta_e) u_e and
    dL/df = lambda."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, f: torch.Tensor, solver: Solver):
        scale = torch.exp(theta.detach().to(torch.float64))
        solver.update_coefficients(scale)
        u, _ = solver.solve(f.detach())
        ctx.solver = solver
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        solver = ctx.solver
        (u,) = ctx.saved_tensors
        lam, _ = solver.solve(grad_u.detach().contiguous())
        g_theta = -solver.element_energy(lam, u)
        return g_theta, lam, None
