"""ctypes binding of ``libicl.so``: every C entry point under its C name.

Argument marshalling only - every step of every operation runs in the HIP
library.  Pointers are plain integers (device addresses) and sizes are Python
ints; ``stream`` is a hipStream_t handle (0 = null stream).  Calls return the
library's ``icl_status`` code; ``check()`` turns a non-zero code into IclError.

The library must be built (``python -m paper_1605_06399_amd.build``); loading
fails loudly otherwise - there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libicl.so")

# icl_status
ICL_OK = 0
ICL_ERR_INVALID_VALUE = 1
ICL_ERR_PITCH = 2
ICL_ERR_RADIUS = 3
ICL_ERR_DTYPE = 4
ICL_ERR_ALIAS = 5
ICL_ERR_WORKSPACE = 6
ICL_ERR_NO_DEVICE = 7
ICL_ERR_HIP = 8
ICL_ERR_UNSUPPORTED = 9
ICL_ERR_TUNE_CACHE = 10

# icl_dtype
ICL_F32, ICL_F16, ICL_BF16, ICL_U8 = 0, 1, 2, 3

# icl_border
ICL_BORDER_CLAMP, ICL_BORDER_CONSTANT = 0, 1

# icl_op
(ICL_OP_CONV_SEP, ICL_OP_CONV2D, ICL_OP_HARRIS, ICL_OP_NMS, ICL_OP_CONV_SEP_BATCHED, ICL_OP_BANK_FWD,
 ICL_OP_BANK_BWD_INPUT, ICL_OP_BANK_BWD_FILTER, ICL_OP_SSE_LOSS, ICL_OP_BANK_FWD_SSE, ICL_OP_CONV2D_U8,
 ICL_OP_CORNERS, ICL_OP_CONV3D_SEP, ICL_OP_COUNT) = range(14)

ICL_MAX_RADIUS = 16
ICL_MAX_WINDOW_RADIUS = 7
ICL_MAX_NMS_RADIUS = 7
ICL_MAX_U8_RADIUS = 7
ICL_MAX_U8_SHIFT = 16
ICL_MAX_RADIUS_3D = 7

_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i = ctypes.c_int
_f = ctypes.c_float
_ll = ctypes.c_longlong


class icl_image_desc(ctypes.Structure):
    _fields_ = [("src", _vp), ("dst", _vp), ("src_pitch", _sz), ("dst_pitch", _sz),
                ("width", _i), ("height", _i), ("radius", _i), ("taps_x", _vp), ("taps_y", _vp)]


# icl_math
ICL_MATH_F32, ICL_MATH_F16_SPLIT = 0, 1


class icl_problem(ctypes.Structure):
    _fields_ = [("op", _i), ("dtype", _i), ("radius", _i), ("width", _i), ("height", _i), ("depth", _i),
                ("n", _i), ("f", _i)]


class IclError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = status_string(status) if _lib is not None else str(status)
        super().__init__(f"{what}: icl status {status} ({msg})" if what else f"icl status {status} ({msg})")


_SIGS = {
    "icl_init": ([], _i),
    "icl_status_string": ([_i], ctypes.c_char_p),
    "icl_last_hip_error": ([], _i),
    "icl_version": ([], ctypes.c_char_p),
    "icl_workspace_size": ([_i, _i, _i, _i, _i, _i, _i, ctypes.POINTER(_sz)], _i),
    "icl_conv_sep": ([_vp, _sz, _vp, _sz, _i, _i, _i, _vp, _vp, _i, _vp, _sz, _vp], _i),
    "icl_conv_sep_border": ([_vp, _sz, _vp, _sz, _i, _i, _i, _vp, _vp, _i, _i, _f, _vp, _sz, _vp], _i),
    "icl_conv2d": ([_vp, _sz, _vp, _sz, _i, _i, _i, _vp, _i, _vp], _i),
    "icl_conv2d_border": ([_vp, _sz, _vp, _sz, _i, _i, _i, _vp, _i, _i, _f, _vp], _i),
    "icl_conv2d_u8": ([_vp, _sz, _vp, _sz, _i, _i, _vp, _i, _i, _i, _i, _vp], _i),
    "icl_conv3d_sep": ([_vp, _sz, _sz, _vp, _sz, _sz, _i, _i, _i, _i, _vp, _vp, _vp, _i, _i, _f, _vp, _sz, _vp], _i),
    "icl_harris": ([_vp, _sz, _vp, _sz, _i, _i, _vp, _i, _f, _vp, _sz, _vp], _i),
    "icl_nms": ([_vp, _sz, _vp, _sz, _i, _i, _i, _f, _vp], _i),
    "icl_corners": ([_vp, _sz, _vp, _sz, _i, _i, _vp, _i, _f, _i, _f, _vp, _sz, _vp, _sz, _vp], _i),
    "icl_batch_plan_create": ([ctypes.POINTER(icl_image_desc), _i, _i, ctypes.POINTER(_vp)], _i),
    "icl_conv_sep_batched": ([_vp, _vp], _i),
    "icl_batch_plan_info": ([_vp, ctypes.POINTER(_ll), ctypes.POINTER(_ll)], _i),
    "icl_batch_plan_destroy": ([_vp], None),
    "icl_batch_graph_create": ([_vp, ctypes.POINTER(_vp)], _i),
    "icl_graph_launch": ([_vp, _vp], _i),
    "icl_graph_destroy": ([_vp], None),
    "icl_bank_fwd": ([_vp, _vp, _vp, _i, _i, _i, _i, _i, _vp], _i),
    "icl_bank_bwd_input": ([_vp, _vp, _vp, _i, _i, _i, _i, _i, _vp, _vp], _i),
    "icl_bank_bwd_filter": ([_vp, _vp, _vp, _i, _i, _i, _i, _i, _vp, _vp, _sz, _vp], _i),
    "icl_sse_loss": ([_vp, _vp, _vp, _ll, _vp, _vp, _sz, _vp], _i),
    "icl_bank_fwd_sse": ([_vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp, _sz, _vp], _i),
    "icl_bank_fwd_sse_noalloc": ([_vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp], _i),
    "icl_tune": ([_i, _i, _i, _i, _i, _vp], _i),
    "icl_tune_model": ([_i, _i, _i, _i, _i, _i, _i, ctypes.c_ulonglong, ctypes.POINTER(_i), _vp], _i),
    "icl_perf_model_fit_predict": ([_vp, _vp, _i, _i, _vp, _i, _vp, _i, _i, ctypes.c_ulonglong], _i),
    "icl_tune_save": ([ctypes.c_char_p], _i),
    "icl_tune_load": ([ctypes.c_char_p], _i),
    "icl_tune_clear": ([], None),
    "icl_variant_count": ([_i], _i),
    "icl_variant_name": ([_i, _i], ctypes.c_char_p),
    "icl_force_variant": ([_i, _i], _i),
    "icl_selected_variant": ([_i, _i, _i, _i, _i, ctypes.POINTER(_i)], _i),
    "icl_tune_problem": ([ctypes.POINTER(icl_problem), _vp], _i),
    "icl_selected_variant_problem": ([ctypes.POINTER(icl_problem), ctypes.POINTER(_i)], _i),
    "icl_batch_plan_tune": ([_vp, _vp], _i),
    "icl_batch_plan_variant": ([_vp, ctypes.POINTER(_i)], _i),
    "icl_set_math": ([_i], _i),
    "icl_get_math": ([], _i),
    "icl_variant_arith": ([_i, _i], ctypes.c_char_p),
}

EXPORTED = tuple(_SIGS)

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1605_06399_amd.build` "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(status: int, what: str = "") -> None:
    if status != ICL_OK:
        raise IclError(status, what)


# ----------------------------------------------------------------------------- entry points (same names as C)

def icl_init() -> int:
    return lib().icl_init()


def status_string(status: int) -> str:
    return lib().icl_status_string(status).decode()


icl_status_string = status_string


def icl_last_hip_error() -> int:
    return lib().icl_last_hip_error()


def icl_version() -> str:
    return lib().icl_version().decode()


def icl_workspace_size(op, width, height, n=0, f=0, radius=0, dtype=ICL_F32):
    out = _sz(0)
    st = lib().icl_workspace_size(op, width, height, n, f, radius, dtype, ctypes.byref(out))
    return st, out.value


def icl_conv_sep(src, src_pitch, dst, dst_pitch, width, height, dtype, taps_x, taps_y, radius,
                 workspace=0, workspace_bytes=0, stream=0) -> int:
    return lib().icl_conv_sep(src, src_pitch, dst, dst_pitch, width, height, dtype, taps_x, taps_y, radius,
                              workspace or None, workspace_bytes, stream or None)


def icl_conv_sep_border(src, src_pitch, dst, dst_pitch, width, height, dtype, taps_x, taps_y, radius, border,
                        constant, workspace=0, workspace_bytes=0, stream=0) -> int:
    return lib().icl_conv_sep_border(src, src_pitch, dst, dst_pitch, width, height, dtype, taps_x, taps_y, radius,
                                     border, constant, workspace or None, workspace_bytes, stream or None)


def icl_conv2d(src, src_pitch, dst, dst_pitch, width, height, dtype, taps, radius, stream=0) -> int:
    return lib().icl_conv2d(src, src_pitch, dst, dst_pitch, width, height, dtype, taps, radius, stream or None)


def icl_conv2d_border(src, src_pitch, dst, dst_pitch, width, height, dtype, taps, radius, border, constant,
                      stream=0) -> int:
    return lib().icl_conv2d_border(src, src_pitch, dst, dst_pitch, width, height, dtype, taps, radius, border,
                                   constant, stream or None)


def icl_conv3d_sep(src, src_row_pitch, src_slice_pitch, dst, dst_row_pitch, dst_slice_pitch, width, height, depth,
                   dtype, taps_x, taps_y, taps_z, radius, border=ICL_BORDER_CLAMP, constant=0.0, workspace=0,
                   workspace_bytes=0, stream=0) -> int:
    return lib().icl_conv3d_sep(src, src_row_pitch, src_slice_pitch, dst, dst_row_pitch, dst_slice_pitch, width,
                                height, depth, dtype, taps_x, taps_y, taps_z, radius, border, constant,
                                workspace or None, workspace_bytes, stream or None)


def icl_conv2d_u8(src, src_pitch, dst, dst_pitch, width, height, taps, radius, shift, border=ICL_BORDER_CLAMP,
                  constant=0, stream=0) -> int:
    return lib().icl_conv2d_u8(src, src_pitch, dst, dst_pitch, width, height, taps, radius, shift, border, constant,
                               stream or None)


def icl_harris(src, src_pitch, resp, resp_pitch, width, height, window_taps, window_radius, k,
               workspace=0, workspace_bytes=0, stream=0) -> int:
    return lib().icl_harris(src, src_pitch, resp, resp_pitch, width, height, window_taps, window_radius, k,
                            workspace or None, workspace_bytes, stream or None)


def icl_nms(resp, resp_pitch, mask, mask_pitch, width, height, radius, threshold, stream=0) -> int:
    return lib().icl_nms(resp, resp_pitch, mask, mask_pitch, width, height, radius, threshold, stream or None)


def icl_corners(src, src_pitch, mask, mask_pitch, width, height, window_taps, window_radius, k, nms_radius,
                threshold, resp=0, resp_pitch=0, workspace=0, workspace_bytes=0, stream=0) -> int:
    return lib().icl_corners(src, src_pitch, mask, mask_pitch, width, height, window_taps, window_radius, k,
                             nms_radius, threshold, resp or None, resp_pitch, workspace or None, workspace_bytes,
                             stream or None)


def icl_batch_plan_create(descs, dtype):
    """descs: sequence of icl_image_desc; returns (status, plan handle)."""
    arr = (icl_image_desc * max(len(descs), 1))(*descs)
    out = _vp(0)
    st = lib().icl_batch_plan_create(arr, len(descs), dtype, ctypes.byref(out))
    return st, out.value


def icl_conv_sep_batched(plan, stream=0) -> int:
    return lib().icl_conv_sep_batched(plan, stream or None)


def icl_batch_plan_info(plan):
    t, p = _ll(0), _ll(0)
    st = lib().icl_batch_plan_info(plan, ctypes.byref(t), ctypes.byref(p))
    return st, t.value, p.value


def icl_batch_plan_destroy(plan) -> None:
    lib().icl_batch_plan_destroy(plan)


def icl_batch_graph_create(plan):
    out = _vp(0)
    st = lib().icl_batch_graph_create(plan, ctypes.byref(out))
    return st, out.value


def icl_graph_launch(exec_, stream=0) -> int:
    return lib().icl_graph_launch(exec_, stream or None)


def icl_graph_destroy(exec_) -> None:
    lib().icl_graph_destroy(exec_)


def icl_bank_fwd(x, w, y, n, f, h, wd, radius, stream=0) -> int:
    return lib().icl_bank_fwd(x, w, y, n, f, h, wd, radius, stream or None)


def icl_bank_bwd_input(gy, w, gx, n, f, h, wd, radius, stream=0, scale=0) -> int:
    return lib().icl_bank_bwd_input(gy, w, gx, n, f, h, wd, radius, scale or None, stream or None)


def icl_bank_bwd_filter(gy, x, gw, n, f, h, wd, radius, workspace=0, workspace_bytes=0, stream=0, scale=0) -> int:
    return lib().icl_bank_bwd_filter(gy, x, gw, n, f, h, wd, radius, scale or None, workspace or None,
                                     workspace_bytes, stream or None)


def icl_sse_loss(y, t, gy, count, loss, workspace=0, workspace_bytes=0, stream=0) -> int:
    return lib().icl_sse_loss(y, t, gy or None, count, loss, workspace or None, workspace_bytes, stream or None)


def icl_bank_fwd_sse(x, w, t, y, gy, loss, n, f, h, wd, radius, workspace=0, workspace_bytes=0, stream=0) -> int:
    return lib().icl_bank_fwd_sse(x, w, t, y or None, gy or None, loss, n, f, h, wd, radius, workspace or None,
                                  workspace_bytes, stream or None)


def icl_bank_fwd_sse_noalloc(x, w, t, y, gy, loss, n, f, h, wd, radius, stream=0) -> int:
    return lib().icl_bank_fwd_sse_noalloc(x, w, t, y or None, gy or None, loss, n, f, h, wd, radius, stream or None)


def icl_tune(op, dtype, radius, width, height, stream=0) -> int:
    return lib().icl_tune(op, dtype, radius, width, height, stream or None)


def icl_tune_model(op, dtype, radius, width, height, samples, top_k, seed=0, stream=0):
    """(status, number of candidates timed)."""
    timed = _i(0)
    st = lib().icl_tune_model(op, dtype, radius, width, height, samples, top_k, seed, ctypes.byref(timed),
                              stream or None)
    return st, timed.value


def icl_perf_model_fit_predict(X, y, Xq, hidden=8, iters=2000, seed=0):
    """(status, predictions) for float64 numpy arrays X [n, d], y [n], Xq [nq, d]."""
    import numpy as np
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    Xq = np.ascontiguousarray(Xq, dtype=np.float64)
    n, d = X.shape if X.ndim == 2 else (0, 0)
    yq = np.zeros(Xq.shape[0] if Xq.ndim == 2 else 0, dtype=np.float64)
    st = lib().icl_perf_model_fit_predict(X.ctypes.data if X.size else None, y.ctypes.data if y.size else None, n,
                                          d, Xq.ctypes.data if Xq.size else None, yq.size,
                                          yq.ctypes.data if yq.size else None, hidden, iters, seed)
    return st, yq


def icl_tune_save(path=None) -> int:
    return lib().icl_tune_save(path.encode() if path else None)


def icl_tune_load(path=None) -> int:
    return lib().icl_tune_load(path.encode() if path else None)


def icl_tune_clear() -> None:
    lib().icl_tune_clear()


def icl_variant_count(op) -> int:
    return lib().icl_variant_count(op)


def icl_variant_name(op, index):
    s = lib().icl_variant_name(op, index)
    return s.decode() if s is not None else None


def icl_force_variant(op, index) -> int:
    return lib().icl_force_variant(op, index)


def icl_selected_variant(op, dtype, radius, width, height):
    out = _i(-1)
    st = lib().icl_selected_variant(op, dtype, radius, width, height, ctypes.byref(out))
    return st, out.value


def variant_names(op):
    return [icl_variant_name(op, i) for i in range(icl_variant_count(op))]


def _problem(op, dtype, radius, width, height, depth=1, n=1, f=1):
    return icl_problem(op, dtype, radius, width, height, depth, n, f)


def icl_tune_problem(op, dtype, radius, width, height, depth=1, n=1, f=1, stream=0) -> int:
    q = _problem(op, dtype, radius, width, height, depth, n, f)
    return lib().icl_tune_problem(ctypes.byref(q), stream or None)


def icl_selected_variant_problem(op, dtype, radius, width, height, depth=1, n=1, f=1):
    q = _problem(op, dtype, radius, width, height, depth, n, f)
    out = _i(-1)
    st = lib().icl_selected_variant_problem(ctypes.byref(q), ctypes.byref(out))
    return st, out.value


def icl_batch_plan_tune(plan, stream=0) -> int:
    return lib().icl_batch_plan_tune(plan, stream or None)


def icl_batch_plan_variant(plan):
    out = _i(-1)
    st = lib().icl_batch_plan_variant(plan, ctypes.byref(out))
    return st, out.value


def icl_set_math(mode) -> int:
    return lib().icl_set_math(mode)


def icl_get_math() -> int:
    return lib().icl_get_math()


def icl_variant_arith(op, index):
    s = lib().icl_variant_arith(op, index)
    return s.decode() if s is not None else None
