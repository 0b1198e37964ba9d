"""ctypes binding of ``libfpclbm.so`` (argument marshalling only).

Every function of ``include/fpclbm.h`` is exposed under the same name.  Each
call checks the returned status and raises :class:`FpcError` with the
library's message on failure.  ``torch`` is imported before the library is
loaded so that the library binds to the HIP runtime torch already loaded.
"""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load torch's HIP runtime first)

_PKG = os.path.dirname(os.path.abspath(__file__))
# FPCLBM_LIB may point at another build of the same library (e.g. a variant
# compiled with different tuning macros).
LIB_PATH = os.environ.get("FPCLBM_LIB") or os.path.join(_PKG, "libfpclbm.so")

FPC_OK = 0
FPC_ERR_ARG = -1
FPC_ERR_SIZE = -2
FPC_ERR_HIP = -3
FPC_ERR_UNSTABLE = -4
FPC_ERR_STATE = -5

FPC_D2Q9_D2Q5 = 1
FPC_D3Q27_D3Q7 = 2
FPC_D2Q9_D2Q9 = 3
FPC_D3Q27_D3Q15 = 4
FPC_MODEL_FP = 0
FPC_MODEL_MCM = 1
FPC_THERMAL_OPTION_A = 0
FPC_THERMAL_OPTION_B = 1
FPC_FP64 = 0
FPC_FP32_DEV = 1

FPC_BC_PERIODIC = 0
FPC_BC_NOSLIP_ADIABATIC = 1
FPC_BC_NOSLIP_DIRICHLET = 2
FPC_BC_LID_ADIABATIC = 3
FPC_BC_LID_DIRICHLET = 4
FPC_TREF_AUTO = -2

EXPORTED = (
    "fpc_version", "fpc_last_error", "fpc_params_bytes", "fpc_params_default", "fpc_params_natural", "fpc_params_mixed",
    "fpc_params_conduction_reference", "fpc_storage_reference",
    "fpc_state_bytes", "fpc_create", "fpc_destroy", "fpc_set_stream", "fpc_set_multistep", "fpc_set_multistep_wait_limit",
    "fpc_multistep_launches",
    "fpc_init", "fpc_step", "fpc_step_nusselt", "fpc_step_diagnostics", "fpc_step_from",
    "fpc_get_step", "fpc_macros", "fpc_diagnostics", "fpc_nusselt_local", "fpc_diagnostics_noalloc", "fpc_save", "fpc_load", "fpc_export_fp64",
    "fpc_import_fp64", "fpc_current_buffer", "fpc_nusselt_seed", "fpc_adjoint_step", "fpc_adjoint_init",
)


class FpcError(RuntimeError):
    def __init__(self, code, func, msg):
        super().__init__(f"{func} failed ({code}): {msg}")
        self.code = code


class fpc_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("nz", ctypes.c_int),
        ("omega_f", ctypes.c_double * 27),
        ("omega_g", ctypes.c_double * 15),
        ("cs2_T", ctypes.c_double),
        ("g_beta", ctypes.c_double),
        ("T0", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("dT_ref", ctypes.c_double),
        ("up_axis", ctypes.c_int),
        ("bc", ctypes.c_int * 6),
        ("wall_T", ctypes.c_double * 6),
        ("lid_u", (ctypes.c_double * 3) * 6),
        ("wall_T_profile", ctypes.c_void_p * 6),
        ("T_ref_slope", ctypes.c_double),
        ("T_ref_axis", ctypes.c_int),
        ("model", ctypes.c_int),
        ("thermal_option", ctypes.c_int),
    ]


_lib = None


def library_path():
    return LIB_PATH


def load():
    """Load the built library (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2504_09041_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(fpc_params)
    vp, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "fpc_version": (i, []),
        "fpc_last_error": (ctypes.c_char_p, []),
        "fpc_params_default": (i, [P, i, i, i, i, i]),
        "fpc_params_natural": (i, [P, d, d, d, i, d, d]),
        "fpc_params_mixed": (i, [P, d, d, d, d, i, d, d]),
        "fpc_params_conduction_reference": (i, [P, i]),
        "fpc_storage_reference": (i, [P, ctypes.POINTER(i), dp]),
        "fpc_state_bytes": (i, [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "fpc_create": (i, [P, vp, vp, vp, ctypes.POINTER(vp)]),
        "fpc_destroy": (i, [vp]),
        "fpc_set_stream": (i, [vp, vp]),
        "fpc_set_multistep": (i, [vp, i]),
        "fpc_set_multistep_wait_limit": (i, [vp, ctypes.c_uint]),
        "fpc_multistep_launches": (i, [vp, ctypes.POINTER(ll)]),
        "fpc_init": (i, [vp, vp]),
        "fpc_step": (i, [vp, i]),
        "fpc_step_nusselt": (i, [vp, i, i, d, vp]),
        "fpc_step_diagnostics": (i, [vp, i, i, vp]),
        "fpc_step_from": (i, [vp, vp, vp]),
        "fpc_params_bytes": (ctypes.c_size_t, []),
        "fpc_get_step": (i, [vp, ctypes.POINTER(ll)]),
        "fpc_macros": (i, [vp, vp, vp, vp]),
        "fpc_diagnostics": (i, [vp, i, dp, dp, dp, dp]),
        "fpc_diagnostics_noalloc": (i, [vp, i, vp]),
        "fpc_nusselt_local": (i, [vp, i, vp]),
        "fpc_save": (i, [vp, vp]),
        "fpc_load": (i, [vp, vp, ll]),
        "fpc_export_fp64": (i, [vp, vp]),
        "fpc_import_fp64": (i, [vp, vp, ll]),
        "fpc_current_buffer": (i, [vp, ctypes.POINTER(vp)]),
        "fpc_nusselt_seed": (i, [vp, i, d, vp, vp]),
        "fpc_adjoint_step": (i, [vp, vp, vp, vp, vp, d, ctypes.POINTER(vp)]),
        "fpc_adjoint_init": (i, [vp, vp, vp, vp, d, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.fpc_params_bytes() != ctypes.sizeof(fpc_params):
        raise ImportError(f"{LIB_PATH}: fpc_params is {lib.fpc_params_bytes()} bytes in the library but "
                          f"{ctypes.sizeof(fpc_params)} in this binding (rebuild the library)")
    _lib = lib
    return lib


def last_error():
    return load().fpc_last_error().decode()


def check(rc, func):
    if rc != FPC_OK:
        raise FpcError(rc, func, last_error())
    return rc


def call(name, *args):
    """Call ``name`` and raise FpcError on a non-zero status."""
    return check(getattr(load(), name)(*args), name)
