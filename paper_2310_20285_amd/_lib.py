"""ctypes binding of libitergp.so (the C ABI declared in include/itergp.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  There is no fallback -- loading fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libitergp.so")

IGP_OK, IGP_EINVAL, IGP_ENOMEM, IGP_EDEVICE, IGP_EUNSUPPORTED = 0, -1, -2, -3, -4
IGP_RBF, IGP_MATERN12, IGP_MATERN32, IGP_MATERN52 = 0, 1, 2, 3
IGP_FP64, IGP_FP32, IGP_BF16, IGP_BF16X3 = 0, 1, 2, 3
IGP_W, IGP_W_PINV = 0, 1
IGP_POLICY_CG, IGP_POLICY_UNIT, IGP_POLICY_USER = 0, 1, 2
IGP_RESIDUAL_EXPLICIT, IGP_RESIDUAL_RECURRENCE = 0, 1
(IGP_VIEW_F, IGP_VIEW_V, IGP_VIEW_Q, IGP_VIEW_S, IGP_VIEW_T, IGP_VIEW_RHS,
 IGP_VIEW_X) = range(7)

KIND_CODE = {"rbf": IGP_RBF, "matern12": IGP_MATERN12, "matern32": IGP_MATERN32,
             "matern52": IGP_MATERN52}
PRECISION_CODE = {"fp64": IGP_FP64, "fp32": IGP_FP32, "bf16": IGP_BF16,
                  "bf16x3": IGP_BF16X3}


class KernelParams(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("reserved", ct.c_int32),
                ("lengthscale", ct.c_double), ("outputscale", ct.c_double)]


IGP_LIK_SOFTMAX, IGP_LIK_POISSON, IGP_LIK_GAUSSIAN, IGP_LIK_BLOCK = 0, 1, 2, 3


class SolverConfig(ct.Structure):
    _fields_ = [("policy", ct.c_int32), ("j_max", ct.c_int32), ("rank_limit", ct.c_int32),
                ("recycle", ct.c_int32), ("tol_abs", ct.c_double), ("tol_rel", ct.c_double),
                ("precision", ct.c_int32), ("residual_mode", ct.c_int32),
                ("max_buffer", ct.c_int32), ("likelihood", ct.c_int32),
                ("noise_var", ct.c_double)]


class StepInfo(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("buffer_cols", ct.c_int32),
                ("recycled_cols", ct.c_int32), ("eig_dropped", ct.c_int32),
                ("converged", ct.c_int32), ("breakdown", ct.c_int32),
                ("k_products", ct.c_int32), ("reserved", ct.c_int32),
                ("res_norm", ct.c_double), ("rhs_norm", ct.c_double), ("eta_min", ct.c_double),
                ("rel_change", ct.c_double), ("psi", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Profile(ct.Structure):
    _fields_ = [("kv_launches", ct.c_int64), ("kv_ms", ct.c_double), ("kv_evals", ct.c_double),
                ("kv_flops", ct.c_double), ("step_ms", ct.c_double), ("steps", ct.c_int64),
                ("kv_symmetric", ct.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ct.c_void_p
_I64 = ct.c_int64
_I32 = ct.c_int32
_SZ = ct.c_size_t

SIGNATURES = {
    "igp_last_error": (ct.c_char_p, []),
    "igp_version": (ct.c_char_p, []),
    "glm_kernel_matmul_ws_bytes": (_SZ, [_I64, _I64, _I64, _I64, _I64, _I32]),
    "glm_kernel_matmul": (ct.c_int, [ct.POINTER(KernelParams), _I32, _P, _I64, _P, _I64, _I64, _P,
                                     _I64, _I64, _I64, _P, _I64, ct.c_double, _I32, _P, _SZ,
                                     _P]),
    "glm_kernel_matmul_noalloc_max_bytes": (_SZ, []),
    "glm_kernel_matmul_noalloc": (ct.c_int, [ct.POINTER(KernelParams), _I32, _P, _I64, _P, _I64,
                                             _I64, _P, _I64, _I64, _I64, _P, _I64, ct.c_double,
                                             _I32, _P]),
    "glm_softmax_hessian_apply": (ct.c_int, [_P, _I64, _I64, _P, _I64, _I64, _P, _I64, _I32,
                                             _I32, _P]),
    "itergp_state_bytes": (_SZ, [_I64, _I64, _I64, ct.POINTER(SolverConfig)]),
    "itergp_init": (ct.c_int, [ct.POINTER(_P), ct.POINTER(KernelParams), _I32,
                               ct.POINTER(SolverConfig), _P, _P, _I64, _I64, _I64, _P, _SZ, _P]),
    "itergp_set_user_actions": (ct.c_int, [_P, _P, _I64, _I64]),
    "itergp_set_block_likelihood": (ct.c_int, [_P, _P, _P]),
    "itergp_newton_step": (ct.c_int, [_P, ct.POINTER(StepInfo)]),
    "itergp_compress": (ct.c_int, [_P, _I32, ct.POINTER(_I32)]),
    "itergp_newton_step_begin": (ct.c_int, [_P]),
    "itergp_newton_step_iterate": (ct.c_int, [_P, _I64, ct.POINTER(_I32)]),
    "itergp_newton_step_end": (ct.c_int, [_P, ct.POINTER(StepInfo)]),
    "itergp_predict_ws_bytes": (_SZ, [_P, _I64]),
    "itergp_predict": (ct.c_int, [_P, _P, _I64, _P, _P, _P, _P, _SZ, _P]),
    "itergp_get_view": (ct.c_int, [_P, _I32, ct.POINTER(_P), ct.POINTER(_I64),
                                   ct.POINTER(_I64), ct.POINTER(_I64)]),
    "itergp_destroy": (ct.c_int, [_P]),
    "igp_host_eigh": (ct.c_int, [_I32, _P, _P, _P]),
    "itergp_set_profiling": (ct.c_int, [_P, _I32]),
    "itergp_get_profile": (ct.c_int, [_P, ct.POINTER(Profile)]),
    "itergp_batched_ws_bytes": (_SZ, [ct.POINTER(_P), _I32]),
    "itergp_newton_step_batched": (ct.c_int, [ct.POINTER(_P), _I32, ct.POINTER(StepInfo), _P,
                                              _SZ]),
    "itergp_newton_step_batched_ex": (ct.c_int, [ct.POINTER(_P), _I32, ct.POINTER(StepInfo),
                                                 _P, _SZ, _I32]),
    "itergp_batched_tuning": (ct.c_int, [ct.c_char_p, _SZ]),
    "itergp_batched_tuning_load": (ct.c_int, [ct.c_char_p, ct.POINTER(_I32)]),
}

_LIB = None


IGP_BATCH_DEVICE_CONTROL = 1


class IterGPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"status {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH) -> ct.CDLL:
    """Load the library (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} not found: build it with "
                               "`python -m paper_2310_20285_amd.build`")
        lib = ct.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def check(code: int):
    if code != IGP_OK:
        raise IterGPError(code, load().igp_last_error().decode())
