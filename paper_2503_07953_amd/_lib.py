"""ctypes binding of libmfc355.so (the C ABI in include/mfc355.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Device memory and streams come from PyTorch.  The
library is required: importing the binding on a machine without the built
library raises immediately, and nothing here falls back to CPU code.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfc355.so")

MFC_ABI_VERSION = 5
MFC_WENO_JS, MFC_WENO_Z, MFC_TENO, MFC_WENO_M = 0, 1, 2, 3
MFC_HLLC, MFC_HLL = 0, 1
MFC_LOW_MACH_NONE, MFC_LOW_MACH_THORNBER, MFC_LOW_MACH_CHEN_APC = 0, 1, 2
MFC_MODEL_ALLAIRE, MFC_MODEL_KAPILA = 0, 1
MFC_OK, MFC_ERR_ARG, MFC_ERR_SHAPE, MFC_ERR_UNSUPPORTED = 0, -1, -2, -3
MFC_ERR_HIP, MFC_ERR_NONFINITE, MFC_ERR_ALLOC = -4, -5, -6
MFC_BC_PERIODIC, MFC_BC_EXTRAP, MFC_BC_SLIPWALL = 0, 1, 2
MFC_FP64, MFC_FP32_MIXED = 0, 1


class mfc_problem(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("num_fluids", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("bc_lo", ctypes.c_int32 * 3),
        ("bc_hi", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double * 3),
        ("gamma", ctypes.c_double * 2),
        ("pi_inf", ctypes.c_double * 2),
        ("weno_eps", ctypes.c_double),
        ("weno_variant", ctypes.c_int32),
        ("riemann_solver", ctypes.c_int32),
        ("low_mach", ctypes.c_int32),
        ("model", ctypes.c_int32),
    ]


_P = ctypes.POINTER(mfc_problem)
_V = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int

# name -> (restype, argtypes); every symbol declared in include/mfc355.h
SIGNATURES = {
    "mfc_abi_version": (_I, []),
    "mfc_status_string": (ctypes.c_char_p, [_I]),
    "mfc_num_eqs": (_I, [_P]),
    "mfc_validate": (_I, [_P]),
    "mfc_create": (_I, [_P, ctypes.POINTER(_V)]),
    "mfc_destroy": (_I, [_V]),
    "mfc_last_error": (ctypes.c_char_p, [_V]),
    "mfc_prim_to_cons": (_I, [_V, _V, _V, _V]),
    "mfc_cons_to_prim": (_I, [_V, _V, _V, _V]),
    "mfc_rhs": (_I, [_V, _V, _V, _V]),
    "mfc_max_signal": (_I, [_V, _V, _V, _V]),
    "mfc_step": (_I, [_V, _V, _D, _D, _D, _V, _V]),
    "mfc_step_static": (_I, [_P, _V, _D, _D, _D, _V, _V, _V]),
    "mfc_conserved_sums": (_I, [_V, _V, _V, _V]),
    "mfc_set_grid": (_I, [_V, _I, _V]),
    "mfc_check": (_I, [_V, _V]),
    "mfc_set_timing": (_I, [_V, _I]),
    "mfc_get_timing": (_I, [_V, _V, _V]),
    "mfc_rhs_vjp": (_I, [_V, _V, _V, _V, _I, _V]),
    "mfc_step_vjp": (_I, [_V, _V, _D, _V, _V, _V]),
    "mfc_step_save_stages": (_I, [_V, _V, _D, _V, _V, _V]),
    "mfc_step_vjp_stages": (_I, [_V, _V, _V, _V, _D, _V, _V, _V]),
    "mfc_cons_to_prim_vjp": (_I, [_V, _V, _V, _V, _I, _V]),
    "mfc_prim_to_cons_vjp": (_I, [_V, _V, _V, _V, _I, _V]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def load() -> ctypes.CDLL:
    """Load libmfc355.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    missing = [name for name in SIGNATURES if not hasattr(L, name)]
    if missing:
        raise LibraryMissing(f"{LIB_PATH} lacks {', '.join(missing)}; rebuild it with __graft_entry__.build()")
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if L.mfc_abi_version() != MFC_ABI_VERSION:
        raise LibraryMissing(f"{LIB_PATH} has ABI version {L.mfc_abi_version()}, the binding expects "
                             f"{MFC_ABI_VERSION}; rebuild it with __graft_entry__.build()")
    _lib = L
    return L


def exported_symbols():
    L = load()
    return {name for name in SIGNATURES if hasattr(L, name)}


def status_string(code: int) -> str:
    return load().mfc_status_string(code).decode()


class MfcError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{status_string(code)} ({code}): {msg}")
        self.code = code


def make_problem(ndim, n, num_fluids, dx, gamma, pi_inf, bc_lo, bc_hi, weno_eps=1e-6,
                 precision=MFC_FP64, weno_variant=MFC_WENO_JS, riemann=MFC_HLLC,
                 low_mach=MFC_LOW_MACH_NONE, model=MFC_MODEL_ALLAIRE) -> mfc_problem:
    p = mfc_problem()
    p.abi_version = MFC_ABI_VERSION
    p.ndim = int(ndim)
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    for d in range(3):
        p.n[d] = n[d]
        p.bc_lo[d] = int(bc_lo[d]) if d < len(bc_lo) else MFC_BC_EXTRAP
        p.bc_hi[d] = int(bc_hi[d]) if d < len(bc_hi) else MFC_BC_EXTRAP
        p.dx[d] = float(dx[d]) if d < len(dx) else 1.0
    p.num_fluids = int(num_fluids)
    p.precision = int(precision)
    for i in range(2):
        p.gamma[i] = float(gamma[i] if i < len(gamma) else gamma[0])
        p.pi_inf[i] = float(pi_inf[i] if i < len(pi_inf) else pi_inf[0])
    p.weno_eps = float(weno_eps)
    p.weno_variant = int(weno_variant)
    p.riemann_solver = int(riemann)
    p.low_mach = int(low_mach)
    p.model = int(model)
    return p
