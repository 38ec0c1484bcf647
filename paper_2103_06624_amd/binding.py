"""ctypes binding of libcvbound: the C ABI of include/cvbound.h, same names.

Argument marshalling only; every step of the bound runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcvbound.so")

CV_OK, CV_EINVAL, CV_ESHAPE, CV_ESPLIT, CV_ENOMEM, CV_EDEVICE = 0, -1, -2, -3, -4, -5
CV_LAYER_DENSE, CV_LAYER_CONV2D = 0, 1

_c_float_p = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p


class cv_layer(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("in_c", ctypes.c_int32), ("in_h", ctypes.c_int32), ("in_w", ctypes.c_int32),
                ("out_c", ctypes.c_int32), ("out_h", ctypes.c_int32), ("out_w", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("stride", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("weight", _vp), ("bias", _vp)]


class cv_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class CvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cvbound error {code}: {msg}")
        self.code = code


_lib = None

# name -> (restype, argtypes)
SIGNATURES = {
    "cv_bound_root_bounds": (ctypes.c_int, [ctypes.POINTER(cv_layer), ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp,
                                            _vp, _vp]),
    "cv_bound_root_bounds_sound": (ctypes.c_int, [ctypes.POINTER(cv_layer), ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp,
                                            _vp, _vp]),
    "cv_bound_root_bounds_opt": (ctypes.c_int, [ctypes.POINTER(cv_layer), ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                                                ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_int32, _vp,
                                                _vp, _vp]),
    "cv_bound_init": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(cv_layer), ctypes.c_int32, ctypes.c_int32,
                                     _vp, _vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp,
                                     _vp]),
    "cv_bound_sizes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64)]),
    "cv_bound_alpha_offset": (ctypes.c_int64, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "cv_bound_alpha_init": (ctypes.c_int, [_vp, _vp, _vp]),
    "cv_bound_eval": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "cv_bound_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cv_bound_grad_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cv_bound_upper": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cv_bound_optimize": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp,
                                         _vp, _vp, ctypes.c_int32, _vp, _vp, _vp]),
    "cv_bound_optimize_joint": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                               _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cv_bound_joint_sizes": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64)]),
    "cv_bound_joint_vars": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp]),
    "cv_bound_update": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cv_bound_autotune": (ctypes.c_int, [_vp, _vp]),
    "cv_bound_set_plan": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "cv_bound_set_parts": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "cv_bound_num_tilings": (ctypes.c_int32, []),
    "cv_bound_set_tiling": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "cv_bound_num_conv_variants": (ctypes.c_int32, []),
    "cv_bound_set_conv_variant": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "cv_bound_conv_variant": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "cv_bound_set_sound": (ctypes.c_int, [_vp, ctypes.c_int32, _vp]),
    "cv_bound_set_input_l2": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "cv_bound_set_input_lp": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_float, _vp]),
    "cv_bound_profile": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.POINTER(cv_kernel_stat),
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _vp]),
    "cv_bound_destroy": (None, [_vp]),
    "cv_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libcvbound.so (raises when it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2103_06624_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != CV_OK:
        raise CvError(rc, lib().cv_last_error().decode(errors="replace"))
    return rc


def _fn(name):
    def call(*args):
        return getattr(lib(), name)(*args)

    call.__name__ = name
    return call


cv_bound_root_bounds = _fn("cv_bound_root_bounds")
cv_bound_root_bounds_sound = _fn("cv_bound_root_bounds_sound")
cv_bound_root_bounds_opt = _fn("cv_bound_root_bounds_opt")
cv_bound_init = _fn("cv_bound_init")
cv_bound_sizes = _fn("cv_bound_sizes")
cv_bound_alpha_offset = _fn("cv_bound_alpha_offset")
cv_bound_alpha_init = _fn("cv_bound_alpha_init")
cv_bound_eval = _fn("cv_bound_eval")
cv_bound_grad = _fn("cv_bound_grad")
cv_bound_grad_noalloc = _fn("cv_bound_grad_noalloc")
cv_bound_upper = _fn("cv_bound_upper")
cv_bound_optimize = _fn("cv_bound_optimize")
cv_bound_autotune = _fn("cv_bound_autotune")
cv_bound_set_plan = _fn("cv_bound_set_plan")
cv_bound_set_parts = _fn("cv_bound_set_parts")
cv_bound_num_tilings = _fn("cv_bound_num_tilings")
cv_bound_set_tiling = _fn("cv_bound_set_tiling")
cv_bound_num_conv_variants = _fn("cv_bound_num_conv_variants")
cv_bound_set_conv_variant = _fn("cv_bound_set_conv_variant")
cv_bound_conv_variant = _fn("cv_bound_conv_variant")
cv_bound_set_sound = _fn("cv_bound_set_sound")
cv_bound_set_input_l2 = _fn("cv_bound_set_input_l2")
cv_bound_set_input_lp = _fn("cv_bound_set_input_lp")
cv_bound_optimize_joint = _fn("cv_bound_optimize_joint")
cv_bound_joint_sizes = _fn("cv_bound_joint_sizes")
cv_bound_joint_vars = _fn("cv_bound_joint_vars")
cv_bound_update = _fn("cv_bound_update")
cv_bound_profile = _fn("cv_bound_profile")
cv_bound_destroy = _fn("cv_bound_destroy")
cv_last_error = _fn("cv_last_error")
