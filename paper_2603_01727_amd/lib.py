"""ctypes declarations of the liblowmach C ABI (include/lowmach.h).

Argument marshalling only: every step of the method runs in the HIP library.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblowmach.so")

LM_OK, LM_EINVAL, LM_ENOMEM, LM_EHIP, LM_ENOCONV, LM_ENONFINITE, LM_ESTATE, LM_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "LM_OK", -1: "LM_EINVAL", -2: "LM_ENOMEM", -3: "LM_EHIP", -4: "LM_ENOCONV",
                -5: "LM_ENONFINITE", -6: "LM_ESTATE", -7: "LM_EUNSUPPORTED"}
SIDE = {"periodic": 0, "slip": 1, "noslip": 2, "inflow": 3, "outflow": 4}
LM_FP64, LM_MIXED, LM_MIXED_FLEXIBLE = 0, 1, 2
PRECISION = {"fp64": LM_FP64, "mixed": LM_MIXED, "mixed-flexible": LM_MIXED_FLEXIBLE}
LM_HOST, LM_DEVICE = 0, 1
LM_BETA_ONE, LM_BETA_INV_RHO = 0, 1
LM_LEVEL_PREDICTED = 2


class lm_grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("L", C.c_double * 3), ("bc", (C.c_int * 2) * 3),
                ("faces", C.c_void_p * 3)]


class lm_params(C.Structure):
    _fields_ = [("Re", C.c_double), ("Pr", C.c_double), ("sigma", C.c_double), ("inv_Fr2", C.c_double),
                ("reacting", C.c_int),
                ("S", C.c_double), ("qs", C.c_double), ("eps", C.c_double), ("tol", C.c_double),
                ("Le_F", C.c_double), ("Le_O", C.c_double),
                ("Da_ib", C.c_double), ("p0", C.c_double), ("dt", C.c_double), ("cfl", C.c_double),
                ("precision", C.c_int), ("poisson_rtol", C.c_double), ("poisson_maxit", C.c_int),
                ("mg_nu", C.c_int), ("with_ib", C.c_int), ("with_adjoint", C.c_int), ("poisson_beta", C.c_int),
                ("p0_closed", C.c_int), ("gamma", C.c_double), ("sutherland_C", C.c_double),
                ("dt_tol", C.c_double)]


class lm_fields(C.Structure):
    _fields_ = [("rho", C.c_void_p), ("v", C.c_void_p * 3), ("Z", C.c_void_p), ("H", C.c_void_p),
                ("T", C.c_void_p), ("P", C.c_void_p), ("F", C.c_void_p * 3)]


class lm_ib(C.Structure):
    _fields_ = [("chi", C.c_void_p), ("v_ib", C.c_void_p * 3), ("Z_ib", C.c_void_p), ("H_ib", C.c_void_p),
                ("S_m", C.c_void_p)]


class lm_side_data(C.Structure):
    _fields_ = [("v", C.c_void_p * 3), ("Z", C.c_void_p), ("H", C.c_void_p), ("F", C.c_void_p),
                ("wall", C.c_void_p)]


class lm_step_stats(C.Structure):
    _fields_ = [("steps", C.c_int), ("dt", C.c_double), ("time", C.c_double),
                ("poisson_iters", C.c_int * 2), ("poisson_relres", C.c_double * 2),
                ("compat", C.c_double * 2), ("total_poisson_iters", C.c_longlong), ("p0", C.c_double),
                ("pc_err", C.c_double), ("pc_err_used", C.c_int)]


class lm_adjoint(C.Structure):
    _fields_ = [("H", C.c_void_p), ("v", C.c_void_p * 3), ("F", C.c_void_p * 3), ("rho_prev", C.c_void_p),
                ("R_H", C.c_void_p), ("R_v", C.c_void_p * 3), ("T", C.c_void_p), ("Z", C.c_void_p),
                ("R_Z", C.c_void_p)]


class lm_project_args(C.Structure):
    _fields_ = [("b", C.c_void_p), ("rho", C.c_void_p), ("P", C.c_void_p), ("mem", C.c_int), ("rtol", C.c_double),
                ("iters", C.c_int), ("relres", C.c_double), ("mean_b", C.c_double)]


EXPORTS = {
    "lm_workspace_size": (C.c_int, [C.POINTER(lm_grid), C.POINTER(lm_params), C.POINTER(C.c_size_t)]),
    "lm_init_grid": (C.c_int, [C.POINTER(lm_grid), C.POINTER(lm_params), C.c_void_p, C.c_size_t, C.c_void_p,
                               C.POINTER(C.c_void_p)]),
    "lm_set_fields": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(lm_fields), C.POINTER(lm_ib), C.c_int]),
    "lm_set_side": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(lm_side_data), C.c_int]),
    "lm_step": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(lm_step_stats)]),
    "lm_project": (C.c_int, [C.c_void_p, C.POINTER(lm_project_args)]),
    "lm_get_fields": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(lm_fields), C.c_int]),
    "lm_get_dt": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "lm_bench_kernel": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    "lm_kernel_timing": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "lm_kernel_timing_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "lm_state_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "lm_save_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lm_load_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lm_kinetic_energy": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "lm_adjoint_seed_ke": (C.c_int, [C.c_void_p]),
    "lm_adjoint_set": (C.c_int, [C.c_void_p, C.POINTER(lm_adjoint), C.c_int]),
    "lm_adjoint_get": (C.c_int, [C.c_void_p, C.POINTER(lm_adjoint), C.c_int]),
    "lm_step_adjoint": (C.c_int, [C.c_void_p]),
    "lm_step_levels_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "lm_save_step_levels": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lm_step_adjoint_levels": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lm_adjoint_initial": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p, C.c_int]),
    "lm_project_static": (C.c_int, [C.POINTER(lm_grid), C.POINTER(lm_params), C.c_void_p,
                                    C.POINTER(lm_project_args)]),
    "lm_last_error": (C.c_char_p, [C.c_void_p]),
    "lm_destroy": (None, [C.c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load liblowmach.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run paper_2603_01727_amd.build.build() first")
    # One HIP runtime per process: PyTorch brings its own libamdhip64 (same
    # soname as the one this library links). Loaded first, it serves both;
    # loaded after this library, a second copy would come in beside it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LowMachError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
