"""ctypes loader for libeb.so (the C ABI in include/eb.h).

Importing this module never builds anything: if the shared library is missing the first call
raises, so no caller can silently fall back to another implementation."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeb.so")

EB_OK, EB_EINVAL, EB_EGEOM, EB_ENOCONV, EB_ENAN, EB_EHIP, EB_ENOMEM = 0, -1, -2, -3, -4, -5, -6
EB_FP64, EB_MIXED = 0, 1
EB_SYS_POISSON, EB_SYS_VISC = 0, 1
EB_OP_HELMHOLTZ, EB_OP_HELMHOLTZ_H, EB_OP_TRANSPOSE = 0, 1, 2
EB_SWITCH_OFF, EB_SWITCH_RECORD, EB_SWITCH_REPLAY = 0, 1, 2
ERRNAMES = {0: "EB_OK", -1: "EB_EINVAL", -2: "EB_EGEOM", -3: "EB_ENOCONV", -4: "EB_ENAN",
            -5: "EB_EHIP", -6: "EB_ENOMEM"}


class EbBox(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("h", C.c_double), ("lo", C.c_double * 3),
                ("periodic", C.c_int * 3), ("wall_u", (C.c_double * 3) * 6)]


class EbBody(C.Structure):
    _fields_ = [("kind", C.c_int), ("center", C.c_double * 3), ("radii", C.c_double * 3),
                ("euler_zyx", C.c_double * 3), ("zlo", C.c_double), ("zhi", C.c_double),
                ("plane_n", C.c_double * 3), ("plane_d", C.c_double), ("u_eb", C.c_double * 3)]


class EbRheology(C.Structure):
    _fields_ = [("law", C.c_int), ("mu", C.c_double), ("tau0", C.c_double),
                ("eps", C.c_double), ("rho", C.c_double), ("kappa", C.c_double),
                ("n", C.c_double), ("eta0", C.c_double)]


class EbStepOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("rtol_visc", C.c_double), ("rtol_mac", C.c_double),
                ("rtol_proj", C.c_double), ("max_iter", C.c_int), ("nu1", C.c_int),
                ("nu2", C.c_int), ("nbottom", C.c_int), ("force", C.c_double * 3),
                ("projection", C.c_int)]


EB_PROJ_CELL, EB_PROJ_NODAL = 0, 1


class EbStepStats(C.Structure):
    _fields_ = [("it_mac", C.c_int * 2), ("it_visc", C.c_int * 2), ("it_proj", C.c_int * 2),
                ("div_proj", C.c_double * 2), ("vcycles", C.c_int), ("status", C.c_int),
                ("fp64_fallbacks", C.c_int), ("dt_stable", C.c_double)]


_P = C.c_void_p
_D = C.c_double
_I = C.c_int
_IP = C.POINTER(C.c_int)
_DP = C.POINTER(C.c_double)

SIGNATURES = {
    "eb_workspace_bytes": (C.c_size_t, [_P, _P]),
    "eb_geometry_build": (_I, [_P, _P, _P, C.c_size_t, C.POINTER(_P), _P]),
    "eb_ctx_destroy": (None, [_P]),
    "eb_ctx_info": (_I, [_P, _IP, _IP, _IP]),
    "eb_ctx_set_graphs": (_I, [_P, _I]),
    "eb_switch_bytes": (C.c_size_t, [_P]),
    "eb_stable_dt": (_I, [_P, _P, _P, _P, _P, _D, _DP, _P]),
    "eb_ctx_set_switches": (_I, [_P, _I, _P, C.c_size_t]),
    "eb_geometry_export": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "eb_apparent_viscosity": (_I, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "eb_viscous_apply": (_I, [_P, _I, _D, _D, _P, _P, _P, _P, _P]),
    "eb_mg_vcycle": (_I, [_P, _I, _I, _D, _D, _D, _P, _P, _P, _P, _P, _P]),
    "eb_mg_sweep": (_I, [_P, _I, _I, _I, _P, _P, _P]),
    "eb_visc_solve": (_I, [_P, _D, _D, _P, _P, _P, _P, _D, _P, _IP, _P]),
    "eb_mac_project": (_I, [_P, _D, _P, _P, _P, _P, _D, _P, _DP, _IP, _P]),
    "eb_cc_project": (_I, [_P, _D, _P, _P, _D, _P, _DP, _IP, _P]),
    "eb_derived": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _IP, _P]),
    "eb_rk2_step": (_I, [_P, _P, _P, _D, _P, _P, _P, _P, _P]),
    "eb_drag": (_I, [_P, _P, _P, _P, _P, _DP, _P]),
    "eb_drag_noalloc": (_I, [_P, _P, _P, _P, _P, _DP, _P]),
    "eb_drag_nodal": (_I, [_P, _P, _P, _P, _P, _DP, _P]),
    "eb_nodal_project": (_I, [_P, _D, _P, _P, _D, _P, _DP, _IP, _P]),
    "eb_pressure_gradient": (_I, [_P, _P, _P, _P]),
    "eb_tape_bytes": (C.c_size_t, [_P]),
    "eb_rk2_step_taped": (_I, [_P, _P, _P, _D, _P, _P, _P, _P, _P, _P]),
    "eb_rk2_step_adjoint": (_I, [_P, _P, _P, _D, _P, _P, _P, _P, _P, _P, _P, _DP, _P, _P]),
    "eb_drag_adjoint": (_I, [_P, _P, _P, _P, _DP, _P, _P, _P, _P, _DP, _P]),
    "eb_mac_project_adjoint": (_I, [_P, _D, _P, _P, _P, _D, _P, _IP, _P]),
    "eb_cc_project_adjoint": (_I, [_P, _D, _P, _P, _D, _P, _IP, _P]),
    "eb_visc_solve_adjoint": (_I, [_P, _D, _D, _P, _P, _P, _P, _D, _P, _P, _P, _P, _IP, _P]),
    "eb_derived_adjoint": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _IP, _P]),
    "eb_last_error": (C.c_char_p, []),
}

_lib = None


class EbError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: {ERRNAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_1905_07392_amd.build.build() "
                "(hipcc --offload-arch=gfx950); there is no fallback implementation")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code, where):
    if code != EB_OK:
        msg = lib().eb_last_error().decode(errors="replace")
        raise EbError(code, where, msg)
    return code
