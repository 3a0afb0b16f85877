"""ctypes declarations of the C ABI in include/gmcp.h (argument marshalling only).

Loads the in-tree ``libgmcp.so``; raises if it has not been built - there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmcp.so")

GMCP_OK, GMCP_E_ARG, GMCP_E_CAPACITY, GMCP_E_PENETRATION = 0, 1, 2, 3
GMCP_E_DEGENERATE, GMCP_E_NONFINITE, GMCP_E_HIP, GMCP_E_TIMEOUT = 4, 5, 6, 7
GMCP_F64, GMCP_KINEMATIC_MASTER, GMCP_MORTAR, GMCP_FEATURES = 1, 2, 4, 8

P = C.c_void_p
i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)


class Layout(C.Structure):
    _fields_ = [("n_env", C.c_int32),
                ("slave_v_off", i32p), ("slave_t_off", i32p),
                ("master_v_off", i32p), ("master_t_off", i32p),
                ("rule_n", i32p), ("kappa", f64p), ("dhat", f64p), ("delta_T", f64p),
                ("cell", f64p), ("flags", C.c_uint32),
                ("kappa_edge", f64p), ("kappa_point", f64p), ("delta_e", f64p)]


class Caps(C.Structure):
    _fields_ = [("grid_cells", C.c_int64), ("grid_items", C.c_int64), ("candidates", C.c_int64),
                ("active", C.c_int64), ("pairs", C.c_int64), ("row_entries", C.c_int64)]


class StatusInfo(C.Structure):
    _fields_ = [("code", C.c_int32), ("reserved", C.c_int32), ("index", C.c_int64),
                ("n_active", C.c_int64), ("n_pairs", C.c_int64), ("nnzb", C.c_int64),
                ("n_candidates", C.c_int64), ("n_swept", C.c_int64), ("need", Caps)]


class Tuning(C.Structure):
    _fields_ = [("query_blocks", C.c_int32), ("light_row_bound", C.c_int32), ("light_row_blocks", C.c_int32),
                ("heavy_row_blocks", C.c_int32)]


class Bsr(C.Structure):
    _fields_ = [("row_ptr", P), ("col", P), ("val", P), ("cap_nnzb", C.c_int64)]


EXPORTS = ["gmcp_workspace_size", "gmcp_create", "gmcp_destroy", "gmcp_set_stream", "gmcp_set_tuning",
           "gmcp_get_tuning",
           "gmcp_build_samples", "gmcp_num_samples", "gmcp_broadphase", "gmcp_assemble",
           "gmcp_ccd_step", "gmcp_ccd_swept", "gmcp_ccd_finish", "gmcp_hvp", "gmcp_energy_frozen", "gmcp_sample_results", "gmcp_pairs", "gmcp_candidates", "gmcp_status",
           "gmcp_strerror", "gmcp_profile", "gmcp_profile_stages", "gmcp_profile_stage_name",
           "gmcp_profile_read", "gmcp_rule", "gmcp_row_classes"]
# include/gmcp_mlp.h
MLP_EXPORTS = ["gmcp_mlp_param_count", "gmcp_mlp_work_bytes", "gmcp_mlp_forward", "gmcp_mlp_backward",
               "gmcp_mlp_mse", "gmcp_mlp_mse_noalloc", "gmcp_mlp_mse_noalloc_max_rows", "gmcp_mlp_adam",
               "gmcp_gemm_bf16"]
# include/gmcp_fem.h
FEM_EXPORTS = ["gmcp_fem_workspace_size", "gmcp_fem_create", "gmcp_fem_destroy", "gmcp_fem_constrain",
               "gmcp_fem_set_stream",
               "gmcp_fem_nnzb", "gmcp_fem_stiffness", "gmcp_fem_energy", "gmcp_fem_apply", "gmcp_fem_solve"]

# include/gmcp_dualmesh.h
DUALMESH_EXPORTS = ["gmcp_dualmesh_embed", "gmcp_dualmesh_update"]

_lib = None


class NativeMissing(RuntimeError):
    pass


def lib():
    """The loaded library; raises NativeMissing if libgmcp.so was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NativeMissing(f"{LIB_PATH} not found: run `python -m paper_2605_24339_amd.build` "
                                "(there is no non-HIP fallback)")
        L = C.CDLL(LIB_PATH)
        L.gmcp_workspace_size.restype = C.c_size_t
        L.gmcp_workspace_size.argtypes = [C.POINTER(Layout), C.POINTER(Caps)]
        L.gmcp_create.restype = C.c_int
        L.gmcp_create.argtypes = [C.POINTER(P), C.POINTER(Layout), C.POINTER(Caps), P, P, P, C.c_size_t, P]
        L.gmcp_destroy.restype = None
        L.gmcp_destroy.argtypes = [P]
        L.gmcp_set_stream.restype = C.c_int
        L.gmcp_set_stream.argtypes = [P, P]
        L.gmcp_build_samples.restype = C.c_int
        L.gmcp_build_samples.argtypes = [P, P, P]
        L.gmcp_num_samples.restype = C.c_int64
        L.gmcp_num_samples.argtypes = [P]
        L.gmcp_broadphase.restype = C.c_int
        L.gmcp_broadphase.argtypes = [P, P, P]
        L.gmcp_assemble.restype = C.c_int
        L.gmcp_assemble.argtypes = [P, P, P, P, P, P, P, C.POINTER(Bsr)]
        L.gmcp_ccd_step.restype = C.c_int
        L.gmcp_ccd_step.argtypes = [P, P, P, P, P, P]
        L.gmcp_ccd_swept.restype = C.c_int
        L.gmcp_ccd_swept.argtypes = [P, P, P, P, P]
        L.gmcp_ccd_finish.restype = C.c_int
        L.gmcp_ccd_finish.argtypes = [P, P, P, P]
        L.gmcp_hvp.restype = C.c_int
        L.gmcp_hvp.argtypes = [P, P, P, P, P]
        L.gmcp_energy_frozen.restype = C.c_int
        L.gmcp_energy_frozen.argtypes = [P, P, P, P]
        L.gmcp_sample_results.restype = C.c_int
        L.gmcp_sample_results.argtypes = [P, P, P, P, P, P, P]
        L.gmcp_set_tuning.restype = C.c_int
        L.gmcp_set_tuning.argtypes = [P, C.POINTER(Tuning)]
        L.gmcp_get_tuning.restype = C.c_int
        L.gmcp_get_tuning.argtypes = [P, C.POINTER(Tuning)]
        L.gmcp_pairs.restype = C.c_int
        L.gmcp_pairs.argtypes = [P, P, P, C.c_int64]
        L.gmcp_candidates.restype = C.c_int
        L.gmcp_candidates.argtypes = [P, P, P, C.c_int64]
        L.gmcp_status.restype = C.c_int
        L.gmcp_status.argtypes = [P, C.POINTER(StatusInfo)]
        L.gmcp_strerror.restype = C.c_char_p
        L.gmcp_strerror.argtypes = [C.c_int]
        L.gmcp_rule.restype = C.c_int
        L.gmcp_rule.argtypes = [C.c_int, C.POINTER(C.c_double)]
        L.gmcp_row_classes.restype = C.c_int
        L.gmcp_row_classes.argtypes = [P, C.POINTER(C.c_int64), P]
        L.gmcp_profile.restype = C.c_int
        L.gmcp_profile.argtypes = [P, C.c_int]
        L.gmcp_profile_stages.restype = C.c_int
        L.gmcp_profile_stages.argtypes = []
        L.gmcp_profile_stage_name.restype = C.c_char_p
        L.gmcp_profile_stage_name.argtypes = [C.c_int]
        L.gmcp_profile_read.restype = C.c_int
        L.gmcp_profile_read.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().gmcp_strerror(int(code)).decode()
