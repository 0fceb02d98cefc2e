"""ctypes binding of liblidkrylov.so (argument marshalling only).

Every computation runs in the HIP library; this module only checks shapes and
passes device pointers.  Importing it fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblidkrylov.so")

LC_OK, LC_ENOTCONV, LC_EINVAL, LC_ESTATE, LC_EHIP, LC_ENOMEM = 0, 1, -1, -2, -3, -4
UNIFORM, SINE, TANH = 0, 1, 2
FP64, MIXED, LEARNED = 0, 1, 2
NOALLOC_MAX_N = 1 << 36  # LC_NOALLOC_MAX_N


class LidKrylovError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lidkrylov error {code}: {msg}")
        self.code = code


class CriticalOpts(C.Structure):
    """lc_critical_opts (field meaning in include/lidkrylov.h)."""
    _fields_ = [("re_tol", C.c_double), ("max_evals", C.c_int), ("newton_tol", C.c_double),
                ("newton_steps", C.c_int), ("lin_tol", C.c_double), ("gmres_m", C.c_int),
                ("max_vectors", C.c_long), ("k", C.c_int), ("m", C.c_int), ("eig_tol", C.c_double),
                ("max_restarts", C.c_int), ("seed", C.c_ulonglong), ("warm_start", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("rho", C.c_double), ("rho0", C.c_double),
                ("rho_hist", C.c_double * 16), ("ms_total", C.c_double), ("guess_used", C.c_int),
                ("guess_eps", C.c_double), ("ms_stencil", C.c_double), ("ms_poisson", C.c_double),
                ("ms_update", C.c_double), ("ms_network", C.c_double)]

    def as_dict(self):
        n = min(self.iterations, 16)
        return {"iterations": self.iterations, "rho": self.rho, "rho0": self.rho0,
                "rho_hist": [self.rho_hist[q] for q in range(n)], "ms_total": self.ms_total,
                "guess_used": bool(self.guess_used), "guess_eps": self.guess_eps,
                "ms_stencil": self.ms_stencil, "ms_poisson": self.ms_poisson, "ms_update": self.ms_update,
                "ms_network": self.ms_network}


_P = C.c_void_p
_D = C.c_double
_I = C.c_int
_SIGS = {
    "lc_version": (C.c_char_p, []),
    "lc_last_error": (C.c_char_p, [_P]),
    "lc_create": (_I, [C.POINTER(_P), _I, _I, _I, _P]),
    "lc_create_in": (_I, [C.POINTER(_P), _I, _I, _I, _P, C.c_size_t, _P]),
    "lc_workspace_query": (_I, [_I, _I, _I, _I, C.POINTER(C.c_size_t)]),
    "lc_destroy": (_I, [_P]),
    "lc_set_stream": (_I, [_P, _P]),
    "lc_vel_size": (C.c_size_t, [_P]),
    "lc_cell_size": (C.c_size_t, [_P]),
    "lc_set_grid": (_I, [_P, _P, _P, _P]),
    "lc_set_stretching": (_I, [_P, _I, _D]),
    "lc_get_grid": (_I, [_P, _P, _P, _P]),
    "lc_set_re": (_I, [_P, _D]),
    "lc_set_lid": (_I, [_P, _D]),
    "lc_set_base_flow": (_I, [_P, _P]),
    "lc_get_base_flow": (_I, [_P, _P, _P]),
    "lc_jacobian_apply": (_I, [_P, _P, _P]),
    "lc_residual": (_I, [_P, _P, _P]),
    "lc_divergence": (_I, [_P, _P, _P, C.POINTER(_D)]),
    "lc_poisson_solve": (_I, [_P, _P, _P, _I]),
    "lc_correct": (_I, [_P, _P, _P, _P, _P]),
    "lc_project": (_I, [_P, _P, _P, _P, _I, _D, _I, C.POINTER(Stats)]),
    "lc_krylov_vector": (_I, [_P, _P, _P, _P, _I, _D, _I, C.POINTER(Stats)]),
    "lc_dot": (_I, [_P, _P, _P, C.POINTER(_D)]),
    "lc_dot_noalloc": (_I, [_P, _P, C.c_size_t, C.POINTER(_D), _P]),
    "lc_axis_modes": (_I, [_I, _P, _P, _P, _P]),
    "lc_hessenberg_eigvals": (_I, [_I, _P, _P, _P]),
    "lc_newton_residual": (_I, [_P, _P, C.POINTER(_D)]),
    "lc_newton_step": (_I, [_P, _D, _I, C.c_long, _I, _D, C.POINTER(_D), C.POINTER(_D), C.POINTER(C.c_long),
                            C.POINTER(_I)]),
    "lc_arnoldi_leading": (_I, [_P, _I, _I, _D, _I, C.c_ulonglong, _P, _I, _D, _P, _P, _P, _P, _P, C.POINTER(_I),
                                C.POINTER(C.c_long)]),
    "lc_critical_re": (_I, [_P, _D, _D, C.POINTER(CriticalOpts), C.POINTER(_D), C.POINTER(_D), _P,
                            C.POINTER(_I)]),
    "lc_net_param_count": (C.c_long, []),
    "lc_net_create": (_I, [C.POINTER(_P), C.c_uint64]),
    "lc_net_destroy": (_I, [_P]),
    "lc_net_last_error": (C.c_char_p, [_P]),
    "lc_net_get_params": (_I, [_P, _P]),
    "lc_net_set_params": (_I, [_P, _P]),
    "lc_net_save": (_I, [_P, C.c_char_p]),
    "lc_net_load": (_I, [_P, C.c_char_p]),
    "lc_net_forward": (_I, [_P, _P, _P, _P, _I, _I, _I]),
    "lc_net_step": (_I, [_P, _P, _P, _P, _I, _I, _I, _D, C.POINTER(_D), _P]),
    "lc_set_net": (_I, [_P, _P]),
    "lc_net_train": (_I, [_P, _P, _I, _D, C.c_uint64, _P]),
    "lc_learned_guess": (_I, [_P, _P, _P, C.POINTER(_D)]),
    "lc_plane_project": (_I, [_P, _P, _I, _P, _P]),
    "lc_set_poisson_method": (_I, [_P, _I]),
    "lc_viscous_solve": (_I, [_P, _P, _P, _D]),
    "lc_stokes_step": (_I, [_P, _P, _P, _D, _I, _D, _I, C.POINTER(Stats)]),
    "lc_stokes_vector": (_I, [_P, _P, _P, _D, _I, _D, _I, C.POINTER(Stats)]),
    "lc_set_stokes_precond": (_I, [_P, _D]),
    "lc_stream_probe": (_I, [_I, C.c_size_t, _I, _P, C.POINTER(_D), C.POINTER(_D)]),
    "lc_profile_enable": (_I, [_P, _I]),
    "lc_profile_read": (_I, [_P, _I, C.POINTER(_D), C.POINTER(C.c_long)]),
    "lc_profile_name": (C.c_char_p, [_I]),
}
KERNEL_CLASSES = ["momentum", "residual", "divergence", "correct", "tp_x", "tp_y", "tp_z", "eigscale",
                  "reduce", "cast", "vector", "nn_forward", "nn_misc", "planes", "tridiag"]

_lib = None


def load():
    """Load the library (once); raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1704_08521_amd.build")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)
