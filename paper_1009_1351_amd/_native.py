"""ctypes binding of libtnlm.so (argument marshalling only).

Every step of the reconstruction runs in the library's HIP kernels; this module
converts torch CUDA tensors to device pointers, fills the C structs of
include/tnlm.h and turns status codes into exceptions. There is no fallback:
if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnlm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1009_1351_amd.build` "
                      "(the HIP library is required; there is no CPU path)")

_lib = C.CDLL(LIB_PATH)

TNLM_OK, TNLM_W_NOT_CONVERGED = 0, 1
INIT_FBP_ALL, INIT_USER = 0, 1
SSD_FP32, SSD_BF16_MFMA, SSD_FP32_SYMMETRIC = 0, 1, 2
SSD_MODES = {"fp32": SSD_FP32, "bf16_mfma": SSD_BF16_MFMA, "fp32_sym": SSD_FP32_SYMMETRIC}


class Geometry(C.Structure):
    _fields_ = [("n_phases", C.c_int32), ("L", C.c_int32), ("pixel_mm", C.c_double), ("n_views", C.c_int32),
                ("n_bins", C.c_int32), ("sad_mm", C.c_double), ("sdd_mm", C.c_double),
                ("dgamma_rad", C.c_double), ("det_offset_bins", C.c_double),
                ("view_angles_rad", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("patch", C.c_int32), ("window", C.c_int32), ("h", C.c_float), ("mu_hat", C.c_float),
                ("beta", C.c_float), ("m1_cgls", C.c_int32), ("m2_jacobi", C.c_int32), ("max_outer", C.c_int32),
                ("tol_rel_update", C.c_float), ("init", C.c_int32), ("ssd_mode", C.c_int32)]


_P = C.c_void_p
_FP = C.POINTER(C.c_float)
for _name, _args, _res in [
    ("tnlm_recon_init", [C.POINTER(_P), C.POINTER(Geometry), C.POINTER(Params), _P], C.c_int),
    ("tnlm_destroy", [_P], None),
    ("tnlm_step", [_P, _P, _P, _P], C.c_int),
    ("tnlm_solve", [_P, _P, _P, _P, C.POINTER(C.c_int32), _FP], C.c_int),
    ("tnlm_get_history", [_P, _FP, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    ("tnlm_project", [_P, _P, _P], C.c_int),
    ("tnlm_backproject", [_P, _P, _P], C.c_int),
    ("tnlm_fbp", [_P, _P, _P, C.c_int32], C.c_int),
    ("tnlm_data_step", [_P, _P, _P, _P, _P], C.c_int),
    ("tnlm_regularize", [_P, _P, _P, _P, _P, C.c_int32], C.c_int),
    ("tnlm_regularize_noalloc", [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_float, _P, _P, _P, _P,
                                 C.c_int32, _P], C.c_int),
    ("tnlm_timing_enable", [_P, C.c_int32], C.c_int),
    ("tnlm_timing_read", [_P, C.POINTER(C.c_double), C.POINTER(C.c_int32)], C.c_int),
    ("tnlm_autotune", [_P, C.POINTER(C.c_int32), _FP], C.c_int),
    ("tnlm_batch_init", [C.POINTER(_P), C.c_int32, C.POINTER(Geometry), C.POINTER(Params), _P], C.c_int),
    ("tnlm_batch_destroy", [_P], None),
    ("tnlm_batch_solve", [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.POINTER(C.c_int32), _FP,
                          C.POINTER(C.c_int)], C.c_int),
    ("tnlm_batch_solve_active", [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), _FP, C.POINTER(C.c_int)], C.c_int),
    ("tnlm_batch_timing_enable", [_P, C.c_int32], C.c_int),
    ("tnlm_batch_timing_read", [_P, C.POINTER(C.c_double), C.POINTER(C.c_int32)], C.c_int),
    ("tnlm_data_cost", [_P, _P, _P, _P, C.POINTER(C.c_double)], C.c_int),
    ("tnlm_cost", [_P, _P, _P, _P, _P, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    ("tnlm_rel_change", [_P, _P, _P, C.POINTER(C.c_double)], C.c_int),
    ("tnlm_set_guide", [_P, _P], C.c_int),
    ("tnlm_image_upsample", [_P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P], C.c_int),
    ("tnlm_cnn_create", [C.POINTER(_P), C.c_int32, C.c_int32, C.c_uint64, C.c_float, _P], C.c_int),
    ("tnlm_cnn_destroy", [_P], None),
    ("tnlm_cnn_num_params", [_P], C.c_int64),
    ("tnlm_cnn_get_params", [_P, _FP, C.c_int64], C.c_int),
    ("tnlm_cnn_set_params", [_P, _FP, C.c_int64], C.c_int),
    ("tnlm_cnn_forward", [_P, _P, _P, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    ("tnlm_cnn_forward_resampled", [_P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    ("tnlm_cnn_loss_grad", [_P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double), _FP, C.c_int64],
     C.c_int),
    ("tnlm_cnn_train_step", [_P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.POINTER(C.c_double)],
     C.c_int),
    ("tnlm_cnn_save", [_P, C.c_char_p], C.c_int),
    ("tnlm_cnn_load", [_P, C.c_char_p], C.c_int),
    ("tnlm_cnn_last_error", [], C.c_char_p),
    ("tnlm_status_string", [C.c_int], C.c_char_p),
    ("tnlm_last_error", [], C.c_char_p),
]:
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


def exported_symbols():
    return ["tnlm_recon_init", "tnlm_destroy", "tnlm_step", "tnlm_solve", "tnlm_get_history", "tnlm_project",
            "tnlm_backproject", "tnlm_fbp", "tnlm_data_step", "tnlm_regularize", "tnlm_regularize_noalloc", "tnlm_timing_enable",
            "tnlm_timing_read", "tnlm_autotune", "tnlm_batch_init", "tnlm_batch_destroy", "tnlm_batch_solve", "tnlm_batch_solve_active",
            "tnlm_batch_timing_enable", "tnlm_batch_timing_read", "tnlm_data_cost", "tnlm_cost", "tnlm_rel_change", "tnlm_set_guide", "tnlm_image_upsample", "tnlm_cnn_create",
            "tnlm_cnn_destroy", "tnlm_cnn_num_params", "tnlm_cnn_get_params", "tnlm_cnn_set_params",
            "tnlm_cnn_forward", "tnlm_cnn_forward_resampled", "tnlm_cnn_loss_grad", "tnlm_cnn_train_step", "tnlm_cnn_save", "tnlm_cnn_load",
            "tnlm_cnn_last_error", "tnlm_status_string", "tnlm_last_error"]


KIND_NAMES = ["project", "backproject", "regularize", "vector", "fbp", "other"]


class TnlmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"tnlm status {status}: {msg}")
        self.status = status


def check(status: int) -> int:
    if status < 0:
        raise TnlmError(status, _lib.tnlm_last_error().decode())
    return status


def check_cnn(status: int) -> int:
    if status < 0:
        raise TnlmError(status, _lib.tnlm_cnn_last_error().decode())
    return status


lib = _lib
