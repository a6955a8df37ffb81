"""ctypes declarations of the C ABI in include/stau.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libstau.so")
LIB_CHECK_PATH = os.path.join(_PKG, "libstau_check.so")  # the same ABI with the kernels' index checks

STAU_OK = 0
STAU_EINVAL = 1
STAU_ENOMEM = 2
STAU_EHIP = 3
STAU_ESINGULAR = 4
STAU_ESTATE = 5
STAU_EUNSUPPORTED = 6
STAU_ENONFINITE = 7
STAU_EBOUNDS = 8
STAU_FP64 = 0
STAU_MIXED = 1
STAU_DCT_AUTO = 0
STAU_DCT_FFT = 1
STAU_DCT_MATMUL = 2
STAU_SOLVE_AUTO = 0
STAU_SOLVE_FP64 = 1
STAU_SOLVE_REFINED = 2
STAU_FACTORS_AUTO = 0
STAU_FACTORS_BAND = 1

RK_SCHEMES = {"RK111": 1, "RK222": 2, "RK443": 3}

ERRNAMES = {1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ESINGULAR", 5: "ESTATE",
            6: "EUNSUPPORTED", 7: "ENONFINITE", 8: "EBOUNDS"}

# every exported symbol of include/stau.h
EXPORTS = (
    "stau_create_domain", "stau_destroy_domain", "stau_build_pencils", "stau_destroy_pencils",
    "stau_query", "stau_factor", "stau_last_singular_pencil", "stau_step", "stau_initial_state",
    "stau_nonlinear", "stau_solve", "stau_check", "stau_kinetic_energy", "stau_last_error",
    "stau_set_kernel_timing", "stau_read_kernel_timing", "stau_adjoint_step",
    "stau_kinetic_energy_adjoint", "stau_initial_state_adjoint", "stau_step_rk", "stau_lbvp", "stau_evp",
    "stau_coeff_to_grid", "stau_grid_to_coeff", "stau_coeff_to_grid_adjoint", "stau_grid_to_coeff_adjoint",
    "stau_kinetic_energy_noalloc",
)
KERNEL_KINDS = ("z_backward", "x_pass", "z_forward_rhs", "pencil_solve", "pencil_factor", "y_pass")


class DomainDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("Nx", C.c_int64),
                ("Ny", C.c_int64), ("Nz", C.c_int64), ("Lx", C.c_double), ("Ly", C.c_double),
                ("dealias", C.c_double), ("device", C.c_int32), ("dct_method", C.c_int32),
                ("mixed_solve", C.c_int32), ("factor_layout", C.c_int32)]


class RBParamsC(C.Structure):
    _fields_ = [("Ra", C.c_double), ("Pr", C.c_double), ("buoyancy", C.c_double),
                ("b_bottom", C.c_double), ("b_top", C.c_double), ("n_gamma", C.c_int32),
                ("reserved", C.c_int32), ("gamma", C.c_double * 4)]


class StateC(C.Structure):
    _fields_ = [("X", C.c_void_p), ("hist", C.c_void_p), ("iteration", C.c_int64),
                ("dt_prev", C.c_double), ("head", C.c_int32), ("reserved", C.c_int32)]


class AdjStateC(C.Structure):
    _fields_ = [("Xbar", C.c_void_p), ("hbar", C.c_void_p)]


class InfoC(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "Nx", "Ny", "Nz", "Ngx", "Ngy", "Ngz", "Px", "P", "P_active", "S", "ne", "n", "kl", "ku",
        "state_elems", "hist_elems", "workspace_bytes")]


class StauError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"stau error {ERRNAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


_loaded = {}


def load(path: str = LIB_PATH):
    """Load libstau.so (or the check build at LIB_CHECK_PATH); raises if it
    has not been built (no fallback)."""
    global _lib
    if path in _loaded:
        return _loaded[path]
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1905_10388_amd/build.py "
                           "(or __graft_entry__.build())")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "stau_create_domain": (i32, [C.POINTER(DomainDesc), C.POINTER(vp)]),
        "stau_destroy_domain": (i32, [vp]),
        "stau_build_pencils": (i32, [vp, C.POINTER(RBParamsC), C.POINTER(vp)]),
        "stau_destroy_pencils": (i32, [vp]),
        "stau_query": (i32, [vp, C.POINTER(InfoC)]),
        "stau_factor": (i32, [vp, dbl, dbl, vp]),
        "stau_last_singular_pencil": (i64, [vp]),
        "stau_step": (i32, [vp, C.POINTER(StateC), dbl, vp]),
        "stau_step_rk": (i32, [vp, i32, dbl, vp, vp]),
        "stau_lbvp": (i32, [vp, vp, vp, vp]),
        "stau_evp": (i32, [vp, dbl, i32, i32, i32, dbl, vp, vp, vp, vp, vp, vp]),
        "stau_initial_state": (i32, [vp, vp, vp, vp]),
        "stau_nonlinear": (i32, [vp, vp, vp, vp]),
        "stau_solve": (i32, [vp, vp, vp, vp]),
        "stau_check": (i32, [vp, vp, vp]),
        "stau_kinetic_energy": (i32, [vp, vp, C.POINTER(dbl), vp]),
        "stau_last_error": (C.c_char_p, []),
        "stau_set_kernel_timing": (i32, [vp, i32]),
        "stau_adjoint_step": (i32, [vp, vp, i64, dbl, dbl, C.POINTER(AdjStateC), vp]),
        "stau_kinetic_energy_adjoint": (i32, [vp, vp, vp, vp]),
        "stau_initial_state_adjoint": (i32, [vp, vp, vp, vp]),
        "stau_read_kernel_timing": (i32, [vp, C.POINTER(dbl), C.POINTER(i64), i32]),
        "stau_kinetic_energy_noalloc": (i32, [vp, vp, vp, vp]),
        "stau_coeff_to_grid": (i32, [vp, vp, C.c_uint32, dbl, vp, vp]),
        "stau_grid_to_coeff": (i32, [vp, vp, C.c_uint32, dbl, vp, vp]),
        "stau_coeff_to_grid_adjoint": (i32, [vp, vp, C.c_uint32, dbl, vp, vp]),
        "stau_grid_to_coeff_adjoint": (i32, [vp, vp, C.c_uint32, dbl, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _loaded[path] = lib
    if path == LIB_PATH:
        _lib = lib
    return lib


def check(rc: int, lib=None):
    """Raise StauError for a nonzero status, with the message of the library
    that returned it (the default one unless lib is given)."""
    if rc != STAU_OK:
        src = lib if lib is not None else _lib
        msg = src.stau_last_error().decode() if src is not None else ""
        raise StauError(rc, msg)
