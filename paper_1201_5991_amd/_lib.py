"""ctypes binding of libmlbddc.so (argument marshalling only).

Every numerical step runs inside the HIP library; this module converts
Python / torch arguments to the C ABI declared in include/mlbddc.h and
raises on error statuses.  It fails loudly when the library is missing.
"""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlbddc.so")

MLBDDC_FP64, MLBDDC_MIXED = 0, 1
MLBDDC_CORNERS, MLBDDC_EDGES, MLBDDC_FACES, MLBDDC_ALL_PRIMAL = 1, 2, 4, 8
MLBDDC_W_STIFFNESS, MLBDDC_W_MULTIPLICITY = 0, 1
MLBDDC_POISSON_Q1, MLBDDC_ELASTICITY_HEX8 = 0, 1

STATUS = {
    0: "OK", -1: "E_ARG", -2: "E_HIP", -3: "E_NOMEM", -4: "E_STATE", -5: "E_NOT_SPD",
    -6: "E_SINGULAR_CONSTRAINTS", -7: "E_NOT_CONVERGED", -8: "E_BREAKDOWN", -9: "E_NO_DEVICE",
}

EXPORTED = [
    "mlbddc_status_string", "mlbddc_default_options", "mlbddc_create", "mlbddc_setup",
    "mlbddc_update_coefficients", "mlbddc_num_dofs", "mlbddc_interface_size", "mlbddc_coarse_size",
    "mlbddc_num_subdomains", "mlbddc_apply", "mlbddc_apply_schur", "mlbddc_condense", "mlbddc_solve",
    "mlbddc_element_energy", "mlbddc_get_coarse_matrix", "mlbddc_destroy", "mlbddc_last_error",
    "mlbddc_element_matrix", "mlbddc_element_load", "mlbddc_plan_counts", "mlbddc_plan_interface",
    "mlbddc_set_profiling", "mlbddc_get_profile", "mlbddc_subdomain_sizes", "mlbddc_assemble_load",
    "mlbddc_interface_dofs", "mlbddc_apply_schur_noalloc",
]
PROF_N = 8
PROF_NAMES = ["update_fp64", "update_fp32", "panel", "diag", "negate", "schur_mv", "precond_mv"]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("rtol", C.c_double), ("max_iter", C.c_int32), ("weights", C.c_int32),
                ("use_graph", C.c_int32), ("panel_tiles", C.c_int32), ("device", C.c_int32),
                ("panel_tiles_precond", C.c_int32), ("tune_table", C.c_char_p), ("lookahead", C.c_int32),
                ("side_stream", C.c_int32), ("stage_cols", C.c_int32), ("mv_group_tiles", C.c_int32),
                ("mfma_f32", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("ndof_per_node", C.c_int32), ("n_nodes", C.c_int64), ("n_elems", C.c_int64),
                ("nodes_per_elem", C.c_int32), ("elem_nodes", C.POINTER(C.c_int32)),
                ("elem_matrix_ref", C.POINTER(C.c_double)), ("elem_scale", C.POINTER(C.c_double)),
                ("dirichlet_nodes", C.POINTER(C.c_uint8))]


class Partition(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("elem_to_sub", C.POINTER(C.c_int32)),
                ("sub_to_parent", C.POINTER(C.POINTER(C.c_int32))), ("constraints", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_res", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double), ("t_plan", C.c_double),
                ("t_setup_num", C.c_double), ("t_solve", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Profile(C.Structure):
    _fields_ = [("time_s", C.c_double * 8), ("flops", C.c_double * 8), ("launches", C.c_int64 * 8),
                ("tiles", C.c_int64 * 8), ("job_time_s", C.c_double * 2), ("panel", C.c_int32 * 2),
                ("bytes", C.c_double * 8), ("stage", C.c_int32 * 2)]

    def as_dict(self):
        d = {n: {"time_s": self.time_s[i], "flops": self.flops[i], "launches": self.launches[i],
                 "tiles": self.tiles[i], "bytes": self.bytes[i]} for i, n in enumerate(PROF_NAMES)}
        d["jobs"] = {"K_time_s": self.job_time_s[0], "M_time_s": self.job_time_s[1],
                     "panel_K": self.panel[0], "panel_M": self.panel[1],
                     "stage_K": self.stage[0], "stage_M": self.stage[1]}
        return d


class ErrorInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("level", C.c_int32), ("subdomain", C.c_int32), ("column", C.c_int32),
                ("message", C.c_char * 256)]


class MlbddcError(RuntimeError):
    def __init__(self, status, info=None):
        self.status = status
        self.name = STATUS.get(status, str(status))
        self.info = info
        msg = self.name
        if info is not None:
            msg += f": {info.message.decode(errors='replace')} (level {info.level}, subdomain {info.subdomain}, column {info.column})"
        super().__init__(msg)


_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1201_5991_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, VP = C.POINTER, C.c_int32, C.c_int64, C.c_double, C.c_void_p
    sig = {
        "mlbddc_status_string": (C.c_char_p, [I32]),
        "mlbddc_default_options": (None, [P(Options)]),
        "mlbddc_create": (I32, [P(VP), P(Options), P(Allocator), VP]),
        "mlbddc_setup": (I32, [VP, P(Mesh), P(Partition)]),
        "mlbddc_update_coefficients": (I32, [VP, VP]),
        "mlbddc_num_dofs": (I64, [VP]),
        "mlbddc_interface_size": (I64, [VP]),
        "mlbddc_coarse_size": (I64, [VP, I32]),
        "mlbddc_num_subdomains": (I64, [VP, I32]),
        "mlbddc_apply": (I32, [VP, VP, VP]),
        "mlbddc_apply_schur": (I32, [VP, VP, VP]),
        "mlbddc_condense": (I32, [VP, VP, VP]),
        "mlbddc_solve": (I32, [VP, VP, VP, VP, P(Stats)]),
        "mlbddc_element_energy": (I32, [VP, VP, VP, VP]),
        "mlbddc_get_coarse_matrix": (I32, [VP, I32, P(D)]),
        "mlbddc_destroy": (I32, [VP]),
        "mlbddc_last_error": (I32, [VP, P(ErrorInfo)]),
        "mlbddc_element_matrix": (I32, [I32, D, D, P(D)]),
        "mlbddc_element_load": (I32, [I32, D, P(D), P(D)]),
        "mlbddc_plan_counts": (I32, [P(Mesh), P(Partition), P(I64)]),
        "mlbddc_plan_interface": (I32, [P(Mesh), P(Partition), P(I64), I32, P(I64), P(I64)]),
        "mlbddc_set_profiling": (I32, [VP, I32]),
        "mlbddc_get_profile": (I32, [VP, P(Profile)]),
        "mlbddc_subdomain_sizes": (I32, [VP, I32, P(I64)]),
        "mlbddc_assemble_load": (I32, [P(Mesh), P(D), P(D), I64]),
        "mlbddc_interface_dofs": (I32, [VP, P(I64)]),
        "mlbddc_apply_schur_noalloc": (I32, [VP, VP, VP]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status, handle=None):
    if status != 0:
        info = ErrorInfo()
        try:
            load().mlbddc_last_error(handle, C.byref(info))
        except Exception:  # pragma: no cover - error path of the error path
            info = None
        raise MlbddcError(status, info)
