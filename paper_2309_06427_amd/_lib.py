"""ctypes declarations of the C ABI in ``include/symstair.h`` (names kept 1:1).

Loading fails loudly when ``libsymstair.so`` has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsymstair.so")

SSP_OK, SSP_ERR_ARG, SSP_ERR_ALLOC, SSP_ERR_HIP, SSP_ERR_STATE = range(5)
SSP_P_OK, SSP_P_NOT_SPD, SSP_P_MAXITER, SSP_P_NONFINITE, SSP_P_BREAKDOWN, SSP_P_INACCURATE = range(6)
SSP_P_WARM_FALLBACK = 8
SSP_P_PC_FALLBACK = 16
SSP_PC_BLOCK_JACOBI, SSP_PC_STAIR_ADD, SSP_PC_SYM_STAIR, SSP_PC_SCALAR_JACOBI, SSP_PC_NEUMANN2, SSP_PC_NEUMANN3 = range(6)
SSP_FP64, SSP_FP32, SSP_FP32_REFINE64 = range(3)

PC = {"bj": SSP_PC_BLOCK_JACOBI, "add": SSP_PC_STAIR_ADD, "sym": SSP_PC_SYM_STAIR,
      "jacobi": SSP_PC_SCALAR_JACOBI, "poly2": SSP_PC_NEUMANN2, "poly3": SSP_PC_NEUMANN3}
PREC = {"fp64": SSP_FP64, "fp32": SSP_FP32, "fp32_refine64": SSP_FP32_REFINE64}

# every symbol the header declares: name -> (restype, argtypes)
_vp, _i32, _i64, _d, _f = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float
_pi32, _pi64 = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
SIGNATURES = {
    "ssp_batch_create": (C.c_int, [_i32, _pi32, _pi32, _pi32, C.c_int, C.POINTER(_vp)]),
    "ssp_batch_destroy": (C.c_int, [_vp]),
    "ssp_layout": (C.c_int, [_vp, _pi64, _pi64, _pi64, _pi64, _pi64]),
    "ssp_kkt_rhs": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ssp_kkt_recover": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ssp_build": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ssp_build_from_blocks": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp, _vp]),
    "ssp_solve": (C.c_int, [_vp, _d, _i32, _vp, _vp, C.c_int, _vp, _vp, _vp, _vp]),
    "ssp_set_keep_inverses": (C.c_int, [_vp, _i32]),
    "ssp_scaled_onchip_horizon": (C.c_int, [_i32, _i32, _i32, _i32, _i32, C.POINTER(C.c_int32)]),
    "ssp_set_reduction_fp64": (C.c_int, [_vp, _i32]),
    "ssp_solve_noalloc": (C.c_int, [_vp, _d, _i32, _vp, _vp, C.c_int, _vp, _vp, _vp, _vp]),
    "ssp_export": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "ssp_solve_outer": (C.c_int, [_vp, _vp, _vp]),
    "ssp_set_mapping": (C.c_int, [_vp, _i32, _i32, _i32]),
    "ssp_mlp_num_params": (_i64, [_i32, _i32]),
    "ssp_mlp_create": (C.c_int, [_i32, _i32, C.c_int, C.POINTER(_vp)]),
    "ssp_mlp_destroy": (C.c_int, [_vp]),
    "ssp_mlp_set_params": (C.c_int, [_vp, _vp, _vp]),
    "ssp_mlp_get_params": (C.c_int, [_vp, _vp, _vp, _vp]),
    "ssp_mlp_set_scaling": (C.c_int, [_vp, _vp, _vp, _f, _vp]),
    "ssp_mlp_get_scaling": (C.c_int, [_vp, _vp, _vp, C.POINTER(_f), _vp]),
    "ssp_mlp_fit_scaling": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "ssp_mlp_predict": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "ssp_mlp_loss_grad": (C.c_int, [_vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp]),
    "ssp_mlp_get_state": (C.c_int, [_vp, _vp, _vp, C.POINTER(C.c_int64), _vp]),
    "ssp_mlp_set_state": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp]),
    "ssp_mlp_adam": (C.c_int, [_vp, _f, _f, _f, _f, _vp]),
    "ssp_gemm_f32": (C.c_int, [_i32, _i32, _i32, _vp, _i32, _i32, _vp, _i32, _i32, _vp, _i32, _vp]),
    "ssp_autotune": (C.c_int, [_vp, _d, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ssp_set_group_mapping": (C.c_int, [_vp, _i32, _i32, _i32]),
    "ssp_get_mapping": (C.c_int, [_vp, _i32, _pi32, _pi32, _pi32, C.POINTER(_f), _pi32]),
    "ssp_solve_kernel": (C.c_int, [_vp, _pi32, _pi32, _pi32]),
    "ssp_set_scaled_mapping": (C.c_int, [_vp, _i32, _i32]),
    "ssp_get_scaled_mapping": (C.c_int, [_vp, _pi32, _pi32, _pi32, C.POINTER(_f)]),
    "ssp_copy_bytes": (C.c_int, [_vp, _vp, _i64, _vp]),
    "ssp_status_str": (C.c_char_p, [C.c_int]),
    "ssp_last_error": (C.c_char_p, []),
}

_lib = None


class SspError(RuntimeError):
    pass


def load() -> C.CDLL:
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SspError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run python -m paper_2309_06427_amd.build_lib)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def check(status: int, what: str) -> None:
    if status != SSP_OK:
        L = load()
        raise SspError(f"{what}: {L.ssp_status_str(status).decode()} ({L.ssp_last_error().decode()})")
