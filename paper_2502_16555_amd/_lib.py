"""ctypes declarations of the C-ABI in include/bte.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbte.so")

BTE_OK, BTE_EINVAL, BTE_EHIP, BTE_ESINGULAR, BTE_ENOCONV, BTE_ENOMEM, BTE_ENONFINITE, BTE_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
PRECISION = {"fp64": 0, "mixed_fp32": 1, "mixed_bf16": 2, "mixed_bf16x3": 3, "fp16_factors": 4}
FIELD = {"const": 0, "rf": 1, "given": 2, "poisson": 3}
VBC = {"natural": 0, "zero_vmax": 1}
KIND = {0: 0, 1: 1, 2: 2}


class bte_process(C.Structure):
    _fields_ = [("kind", C.c_int32), ("threshold_eV", C.c_double), ("mass_ratio", C.c_double),
                ("n_tab", C.c_int32), ("eps_eV", C.POINTER(C.c_double)), ("sigma_m2", C.POINTER(C.c_double))]


class bte_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nr", C.c_int32), ("ntheta", C.c_int32), ("nl", C.c_int32),
                ("v_bc", C.c_int32), ("L_m", C.c_double), ("eps_max_eV", C.c_double), ("T0_K", C.c_double),
                ("dt_s", C.c_double), ("n_proc", C.c_int32), ("proc", C.POINTER(bte_process)),
                ("n_bins", C.c_int32), ("bin_edges_eV", C.POINTER(C.c_double)), ("scal", C.POINTER(C.c_double)),
                ("precision", C.c_int32), ("refine_max_iter", C.c_int32), ("refine_rtol", C.c_double),
                ("field_mode", C.c_int32), ("field_freq_hz", C.c_double), ("field_a1", C.c_double),
                ("poisson_V0", C.c_double), ("n_discharges", C.c_int32), ("nx_per", C.POINTER(C.c_int32)),
                ("n0_per", C.POINTER(C.c_double)), ("E0_per", C.POINTER(C.c_double)), ("x_fp32", C.c_int32)]


class bte_field(C.Structure):
    _fields_ = [("E_half", C.c_void_p), ("ni", C.c_void_p)]


class bte_implicit_opts(C.Structure):
    _fields_ = [("newton_rtol", C.c_double), ("max_newton", C.c_int32), ("gmres_rtol", C.c_double),
                ("restart", C.c_int32), ("max_gmres", C.c_int32), ("precond", C.c_int32)]


class bte_implicit_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("gmres_iters", C.c_int32), ("residual", C.c_double),
                ("residual0", C.c_double)]


class bte_info(C.Structure):
    _fields_ = [("nx_total", C.c_int32), ("n", C.c_int32), ("n_params", C.c_int32), ("n_discharges", C.c_int32),
                ("vmax", C.c_double), ("bytes_device", C.c_double), ("lu_flops_per_step", C.c_double),
                ("q_bytes_per_half_step", C.c_double)]


VSOLVER_LU = 0
VSOLVER_GMRES = 1
VSOLVER_BANDED = 2
VSOLVER_HESSENBERG = 3
TUNE_LU_STREAMS = 0
TUNE_UPDATE_KC = 1
TUNE_FORM_XPB = 2
TUNE_PANEL_PAIRS = 3
TUNE_STATIC_PIVOTING = 4
TUNE_LOOK_AHEAD = 5
TUNE_FORM_OVERLAP = 6
PRECOND_SPLIT = 0
PRECOND_SEMI_IMPLICIT = 1
ION_SCRATCH_DOUBLES = 2097152   # BTE_ION_SCRATCH_DOUBLES

EXPORTS = {
    "bte_setup_operators": (C.c_int, [C.POINTER(bte_config), C.c_int, C.POINTER(C.c_void_p)]),
    "bte_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, bte_field, C.c_void_p]),
    "bte_moments": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bte_moments_vjp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bte_adjoint_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, bte_field, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p]),
    "bte_initial_maxwellian": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "bte_xstep": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "bte_xstep_T": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "bte_vstep": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bte_ion_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "bte_ion_step_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "bte_hybrid_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "bte_implicit_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, bte_implicit_opts,
                                    C.POINTER(bte_implicit_stats), C.c_void_p]),
    "bte_field_eval": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, bte_field, C.c_void_p, C.c_void_p]),
    "bte_get_operator": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "bte_host_operator": (C.c_int, [C.POINTER(bte_config), C.c_int32, C.POINTER(C.c_double)]),
    "bte_get_info": (C.c_int, [C.c_void_p, C.POINTER(bte_info)]),
    "bte_factor_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_int32)]),
    "bte_get_status": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "bte_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "bte_set_refine": (C.c_int, [C.c_void_p, C.c_int32, C.c_double]),
    "bte_get_timing": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "bte_set_tuning": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "bte_graph_capture": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_int32, bte_field]),
    "bte_graph_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "bte_set_vsolver": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                  C.c_double, C.c_int32]),
    "bte_get_tuning": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "bte_destroy": (None, [C.c_void_p]),
    "bte_status_string": (C.c_char_p, [C.c_int]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libbte.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2502_16555_amd.build`")
    # The library and torch must share one HIP runtime (both need the soname
    # libamdhip64.so.7): load torch's copy first so that libbte.so binds to it.
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


class BteError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = load().bte_status_string(code).decode()
        super().__init__(f"{where}: {msg} ({code})")


def check(code: int, where: str):
    if code != BTE_OK:
        raise BteError(code, where)
