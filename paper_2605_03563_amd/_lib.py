"""ctypes declarations of the C ABI in include/poisson.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpoisson_mi355x.so")

OK, WARN_MAXITER = 0, 1
EINVAL, EGRID, EWORKSPACE, EHIP, ENUMERIC, EADMIT, ETIMEOUT = -1, -2, -3, -4, -5, -6, -7

CARTESIAN, SPHERICAL_LOG = 0, 1
SOR, CG, BICGSTAB, MG, MG_IR32, BICGSTAB_MG32, MG_SPAI, MG_SPAI32, PCG = 0, 1, 2, 3, 4, 5, 6, 7, 8
OMEGA_OPT, OMEGA_OPT_A, OMEGA_CHEBYSHEV, OMEGA_FIXED = 0, 1, 2, 3


class Grid(C.Structure):
    _fields_ = [("coord", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("ghost", C.c_int32), ("pad_", C.c_int32),
                ("pitch", C.c_int64 * 2), ("ext_in", C.c_int32), ("ext_out", C.c_int32),
                ("r_pad", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("order", C.c_int32), ("lmax", C.c_int32),
                ("nu1", C.c_int32), ("nu2", C.c_int32), ("coarsest", C.c_int32),
                ("omega_mode", C.c_int32), ("max_iter", C.c_int32), ("check_every", C.c_int32),
                ("pad_", C.c_int32), ("omega", C.c_double), ("four_pi_G", C.c_double),
                ("point_mass", C.c_double), ("coarse_tol", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("status", C.c_int32), ("rel_residual", C.c_double),
                ("b_norm", C.c_double), ("rate", C.c_double), ("t_multipole_ms", C.c_double),
                ("t_iter_ms", C.c_double), ("residual_history", C.POINTER(C.c_double)),
                ("history_cap", C.c_int32), ("history_len", C.c_int32)]


# symbol -> (restype, argtypes)
SIGNATURES = {
    "poisson_default_opts": (None, [C.POINTER(Opts), C.c_int32]),
    "poisson_workspace_bytes": (C.c_size_t, [C.POINTER(Grid), C.POINTER(Opts)]),
    "poisson_plan": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(Grid), C.POINTER(Opts), C.c_void_p,
                               C.c_size_t, C.c_void_p]),
    "multipole_boundary": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                     C.POINTER(C.c_double)]),
    "multipole_boundary_noalloc": (C.c_int, [C.POINTER(Grid), C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                                             C.c_double, C.POINTER(C.c_double), C.c_void_p]),
    "poisson_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Grid), C.c_double,
                                C.POINTER(Stats)]),
    "poisson_plan_set_capture_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "poisson_plan_destroy": (None, [C.c_void_p]),
    "poisson_strerror": (C.c_char_p, [C.c_int]),
    "poisson_last_error": (C.c_char_p, []),
    "poisson_op_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "poisson_op_residual": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_double)]),
    "poisson_op_smooth": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                    C.c_double]),
    "poisson_op_restrict": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "poisson_op_restrict_residual": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "poisson_op_prolong_add": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "poisson_op_vcycle": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "poisson_op_sweep_resident": (C.c_int, [C.c_void_p, C.c_int32]),
    "poisson_op_precond": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "poisson_server_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_void_p, C.c_size_t, C.c_int32,
                                        C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                        C.c_int32, C.c_int32]),
    "poisson_server_submit": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_int64)]),
    "poisson_server_poll": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.POINTER(Stats),
                                      C.POINTER(C.c_double)]),
    "poisson_server_wait": (C.c_int, [C.c_void_p, C.c_int64, C.c_double]),
    "poisson_server_reserve": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "poisson_server_footprint": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_size_t)]),
    "poisson_server_usage": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]),
    "poisson_server_destroy": (None, [C.c_void_p]),
}

_lib = None


def load() -> C.CDLL:
    """Load the gfx950 library; fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2605_03563_amd.build` (there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
