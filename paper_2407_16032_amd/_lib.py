"""ctypes declarations of the C ABI in include/wlmi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwlmi.so")

WL_OK = 0
STATUS = {0: "WL_OK", 1: "WL_ERR_INVALID_ARG", 2: "WL_ERR_WORKSPACE_TOO_SMALL", 3: "WL_ERR_HIP",
          4: "WL_ERR_NONFINITE", 5: "WL_ERR_UNSUPPORTED"}
WL_F32, WL_F64 = 0, 1
BODY_KIND = {"none": 0, "sphere": 1, "box": 2, "grid": 3, "plane": 4}
BODY_OP = {"union": 0, "intersect": 1, "subtract": 2}
FIELDS = {"u": 0, "u0": 1, "f": 2, "V": 3, "mu0": 4, "mu1": 5, "p": 6, "x": 7, "r": 8, "L": 9, "iD": 10,
          "adj_u": 11, "adj_p": 12}

# every symbol include/wlmi.h declares
EXPORTS = ["wl_workspace_bytes", "wl_sim_create", "wl_sim_destroy", "wl_measure_body", "wl_step",
           "wl_apply_bc", "wl_conv_diff", "wl_project", "wl_poisson_solve", "wl_forces", "wl_forces_static", "wl_field",
           "wl_levels", "wl_set_time", "wl_get_time", "wl_sim_time", "wl_profile", "wl_profile_groups", "wl_profile_read", "wl_pg_set_weights",
           "wl_pg_get_weights", "wl_pg_mode", "wl_pg_forward", "wl_pg_train_step", "wl_pg_stats", "wl_body_update",
           "wl_body_box",
           "wl_adj_reset", "wl_adj_forces", "wl_adj_step", "wl_adj_step_cfl", "wl_adj_body_grad", "wl_last_error"]
PG_PARAMS = 8673
KERNELS = ["measure", "coef", "flux", "bdim", "bc", "exit", "divres", "pcg_a", "pcg_b", "restrict",
           "prolong", "project", "cfl", "forces", "coarse", "reduce", "pg_infer", "pg_train", "adjoint"]


class SimDesc(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int64 * 3), ("L", C.c_double), ("U", C.c_double * 3),
                ("nu", C.c_double),
                ("periodic_mask", C.c_uint), ("convective_exit", C.c_int), ("prec", C.c_int),
                ("eps", C.c_double), ("dt0", C.c_double), ("dt_max", C.c_double),
                ("cfl_nu_coef", C.c_double), ("mg_tol", C.c_double), ("mg_itmax", C.c_int),
                ("pcg_iters", C.c_int), ("learned_guess", C.c_int), ("adjoint", C.c_int),
                ("solver_path", C.c_int), ("reduce_mode", C.c_int),
                ("blend_mode", C.c_int), ("vcycle_graph", C.c_int)]


class BodyDesc(C.Structure):
    pass


BodyDesc._fields_ = [("kind", C.c_int), ("center", C.c_double * 3), ("radius", C.c_double),
                     ("half_extent", C.c_double * 3), ("heave_amp", C.c_double), ("pitch_amp", C.c_double),
                     ("freq", C.c_double), ("phase_h", C.c_double), ("phase_p", C.c_double),
                     ("pivot_offset", C.c_double * 3), ("spin_omega", C.c_double),
                     ("velocity", C.c_double * 3), ("heave_dir", C.c_double * 3), ("scale_amp", C.c_double * 3),
                     ("phase_s", C.c_double), ("normal", C.c_double * 3), ("shell", C.c_double),
                     ("sdf_grid", C.c_void_p), ("vel_grid", C.c_void_p), ("grid_n", C.c_int64 * 3),
                     ("grid_origin", C.c_double * 3), ("grid_h", C.c_double), ("op", C.c_int),
                     ("next", C.POINTER(BodyDesc))]


class StepStats(C.Structure):
    _fields_ = [("dt", C.c_double), ("t", C.c_double), ("dt_next", C.c_double), ("vcycles", C.c_int * 2),
                ("res0_linf", C.c_double * 2), ("res_linf", C.c_double * 2), ("res_l2", C.c_double * 2), ("div_linf", C.c_double),
                ("converged", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("vcycles", C.c_int), ("res0_linf", C.c_double), ("res_linf", C.c_double),
                ("res_l2", C.c_double), ("converged", C.c_int)]


_lib = None


class WlError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load the HIP library; raise (never fall back) if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise WlError("libwlmi.so is not built (run __graft_entry__.build()): %s" % path)
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.wl_workspace_bytes.restype = C.c_size_t
    lib.wl_workspace_bytes.argtypes = [C.POINTER(SimDesc), C.POINTER(BodyDesc)]
    lib.wl_sim_create.restype = C.c_int
    lib.wl_sim_create.argtypes = [C.POINTER(SimDesc), C.POINTER(BodyDesc), P, C.c_size_t, P, C.POINTER(P)]
    lib.wl_sim_destroy.restype = C.c_int
    lib.wl_sim_destroy.argtypes = [P]
    lib.wl_measure_body.restype = C.c_int
    lib.wl_measure_body.argtypes = [P, C.c_double]
    lib.wl_step.restype = C.c_int
    lib.wl_step.argtypes = [P, C.c_int, C.POINTER(StepStats)]
    lib.wl_apply_bc.restype = C.c_int
    lib.wl_apply_bc.argtypes = [P]
    lib.wl_conv_diff.restype = C.c_int
    lib.wl_conv_diff.argtypes = [P]
    lib.wl_project.restype = C.c_int
    lib.wl_project.argtypes = [P, C.c_double, C.POINTER(SolveStats)]
    lib.wl_poisson_solve.restype = C.c_int
    lib.wl_poisson_solve.argtypes = [P, P, P, C.c_double, C.c_int, C.POINTER(SolveStats)]
    lib.wl_forces.restype = C.c_int
    lib.wl_forces.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.wl_forces_static.restype = C.c_int
    lib.wl_forces_static.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.wl_field.restype = C.c_int
    lib.wl_field.argtypes = [P, C.c_int, C.c_int, C.POINTER(P), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.wl_levels.restype = C.c_int
    lib.wl_levels.argtypes = [P, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int64)]
    lib.wl_set_time.restype = C.c_int
    lib.wl_set_time.argtypes = [P, C.c_double, C.c_double]
    lib.wl_get_time.restype = C.c_int
    lib.wl_get_time.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.wl_sim_time.restype = C.c_int
    lib.wl_sim_time.argtypes = [P, C.POINTER(C.c_double)]
    lib.wl_profile.restype = C.c_int
    lib.wl_profile.argtypes = [P, C.c_int]
    lib.wl_profile_groups.restype = C.c_int
    lib.wl_profile_groups.argtypes = [P, C.c_uint32]
    lib.wl_profile_read.restype = C.c_int
    lib.wl_profile_read.argtypes = [P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    FP = C.POINTER(C.c_float)
    lib.wl_pg_set_weights.restype = C.c_int
    lib.wl_pg_set_weights.argtypes = [P, FP]
    lib.wl_pg_get_weights.restype = C.c_int
    lib.wl_pg_get_weights.argtypes = [P, FP]
    lib.wl_pg_mode.restype = C.c_int
    lib.wl_pg_mode.argtypes = [P, C.c_int, C.c_double, C.c_int, C.c_int, C.c_uint64]
    lib.wl_pg_forward.restype = C.c_int
    lib.wl_pg_forward.argtypes = [P, P, C.POINTER(C.c_int64), P]
    lib.wl_pg_train_step.restype = C.c_int
    lib.wl_pg_train_step.argtypes = [P, P, P, P, C.POINTER(C.c_int64), FP, C.POINTER(C.c_double), C.c_int]
    lib.wl_pg_stats.restype = C.c_int
    lib.wl_pg_stats.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    DP = C.POINTER(C.c_double)
    lib.wl_body_update.restype = C.c_int
    lib.wl_body_update.argtypes = [P, C.POINTER(BodyDesc)]
    lib.wl_body_box.restype = C.c_int
    lib.wl_body_box.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.wl_adj_reset.restype = C.c_int
    lib.wl_adj_reset.argtypes = [P]
    lib.wl_adj_forces.restype = C.c_int
    lib.wl_adj_forces.argtypes = [P, DP, C.c_double, DP]
    lib.wl_adj_step.restype = C.c_int
    lib.wl_adj_step.argtypes = [P, C.c_double, C.POINTER(StepStats), C.POINTER(SolveStats)]
    lib.wl_adj_step_cfl.restype = C.c_int
    lib.wl_adj_step_cfl.argtypes = [P, C.c_double, C.c_int, DP, C.POINTER(StepStats), C.POINTER(SolveStats)]
    lib.wl_adj_body_grad.restype = C.c_int
    lib.wl_adj_body_grad.argtypes = [P, DP, DP]
    lib.wl_last_error.restype = C.c_char_p
    lib.wl_last_error.argtypes = []
    _lib = lib
    return lib


def check(status: int, what: str):
    if status != WL_OK:
        msg = _lib.wl_last_error().decode() if _lib is not None else ""
        raise WlError("%s failed: %s (%s)" % (what, STATUS.get(status, status), msg))
