"""ctypes declarations of libinvdft.so (the C ABI in include/invdft.h).

Loading fails loudly when the built library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libinvdft.so")

FE_OK, FE_EINVAL, FE_ENOMEM, FE_EDEVICE, FE_ENOCONV, FE_ENOTPD, FE_EGAP, FE_ESTATES = range(8)
FE_F64, FE_F32, FE_BF16 = 0, 1, 2
FE_XC_SLATER, FE_XC_LB94 = 0, 1
(FE_OP_KS_APPLY, FE_OP_CHEB_FILTER, FE_OP_RAYLEIGH_RITZ, FE_OP_ADJOINT_SOLVE, FE_OP_LOSS_GRAD, FE_OP_EIGENSOLVE,
 FE_OP_ALONG_PSI, FE_OP_POISSON, FE_OP_ADJOINT_DEFLATED) = range(9)

STATUS_NAMES = {0: "FE_OK", 1: "FE_EINVAL", 2: "FE_ENOMEM", 3: "FE_EDEVICE", 4: "FE_ENOCONV",
                5: "FE_ENOTPD", 6: "FE_EGAP", 7: "FE_ESTATES"}

vp = C.c_void_p
dp = C.POINTER(C.c_double)
ip = C.POINTER(C.c_int)
i64p = C.POINTER(C.c_int64)

# name -> (restype, argtypes); every symbol declared in include/invdft.h
SIGNATURES = {
    "fe_mesh_create": (C.c_int, [C.c_int, C.c_int, C.c_double, C.POINTER(vp)]),
    "fe_mesh_create_graded": (C.c_int, [C.c_int, C.c_int, dp, C.POINTER(vp)]),
    "fe_mesh_create_mapped": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_double, C.POINTER(vp)]),
    "fe_mesh_info": (C.c_int, [vp, i64p, i64p, ip, dp]),
    "fe_mesh_nodes": (C.c_int, [vp, vp, vp, vp]),
    "fe_mesh_kinetic_diag": (C.c_int, [vp, vp, vp]),
    "fe_mesh_destroy": (C.c_int, [vp]),
    "fe_workspace_bytes": (C.c_size_t, [vp, C.c_int, C.c_int, C.c_int]),
    "fe_last_error": (C.c_char_p, []),
    "ks_apply": (C.c_int, [vp, vp, dp, vp, vp, C.c_int, C.c_int, C.c_int, vp]),
    "cheb_filter": (C.c_int, [vp, vp, C.c_int, C.c_double, C.c_double, C.c_double, vp, C.c_int, C.c_int,
                              C.c_int, vp, vp]),
    "rayleigh_ritz": (C.c_int, [vp, vp, vp, dp, dp, C.c_int, C.c_int, vp, vp]),
    "ks_eigensolve": (C.c_int, [vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                C.c_double, dp, dp, ip, ip, vp, vp]),
    "adjoint_solve": (C.c_int, [vp, vp, vp, dp, C.c_int, vp, vp, C.c_double, C.c_int, ip, dp, C.c_int, vp, vp]),
    "adjoint_solve_deflated": (C.c_int, [vp, vp, vp, dp, C.c_int, vp, dp, C.c_int, vp, vp, C.c_double, C.c_int, ip,
                                         dp, vp, vp]),
    "loss_grad": (C.c_int, [vp, vp, dp, C.c_int, vp, vp, C.c_double, vp, vp, vp, dp, vp, vp]),
    "loss_grad_noalloc": (C.c_int, [vp, vp, dp, C.c_int, vp, vp, C.c_double, vp, vp, vp, dp, vp]),
    "loss_grad_noalloc_max_bytes": (C.c_size_t, []),
    "fe_dot": (C.c_int, [vp, vp, C.c_int64, dp, vp, vp]),
    "fe_axpby": (C.c_int, [C.c_double, vp, C.c_double, vp, C.c_int64, vp]),
    "fe_apply_timing": (C.c_int, [C.c_int]),
    "fe_apply_timing_read": (C.c_int, [C.c_int, i64p, dp, dp, dp]),
    "fe_sweep_timing_read": (C.c_int, [C.c_int, i64p, dp, dp, dp]),
    "vxc_mesh_create": (C.c_int, [vp, C.c_int, dp, C.c_int, dp, C.c_int, dp, C.POINTER(vp)]),
    "vxc_mesh_info": (C.c_int, [vp, i64p, ip]),
    "vxc_mesh_destroy": (C.c_int, [vp]),
    "vxc_prolong": (C.c_int, [vp, vp, vp, vp, vp]),
    "vxc_restrict": (C.c_int, [vp, vp, vp, vp]),
    "poisson_solve": (C.c_int, [vp, vp, C.c_double, vp, C.c_double, C.c_int, ip, dp, dp, vp, vp]),
    "xc_initial_guess": (C.c_int, [vp, vp, vp, C.c_double, C.c_double, C.c_double, C.c_int, vp, vp, vp]),
    "fermi_occupations": (C.c_int, [dp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp, dp,
                                    ip]),
    "adjoint_along_psi": (C.c_int, [vp, vp, C.c_int, dp, C.c_double, C.c_double, C.c_double, vp, vp, vp, dp,
                                    dp, vp, vp]),
}

_lib = None


def load() -> C.CDLL:
    """Load the built library (once). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2510_10529_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FEError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load().fe_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def check(status: int, where: str, allow=()):
    if status != FE_OK and status not in allow:
        raise FEError(status, where)
    return status
