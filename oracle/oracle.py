"""numpy front end of the FP64 CPU oracle (``icl_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this module.  The product path never imports it.

Inputs are promoted to float64 here (float32 and integer images exactly;
binary16 / bfloat16 storage through the oracle's own decoders), every sum runs
in double precision inside the C library, and results come back as float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "icl_oracle.c")
_LIB_DEFAULT = os.path.join(_HERE, "liboracle.so")
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
# ICL_ORACLE_SANITIZED=1 loads the AddressSanitizer + UndefinedBehaviorSanitizer build (the
# process must preload the sanitizer runtime: LD_PRELOAD=$(gcc -print-file-name=libasan.so))
_LIB = _LIB_SAN if os.environ.get("ICL_ORACLE_SANITIZED") == "1" else _LIB_DEFAULT

_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_L = ctypes.POINTER(ctypes.c_long)
_U16 = ctypes.POINTER(ctypes.c_uint16)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_I16 = ctypes.POINTER(ctypes.c_int16)

# boundary conditions (Section 5, Fig. 3)
BORDERS = {"clamp": 0, "constant": 1}


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP for row splitting); with `sanitize`,
    a separate library built with AddressSanitizer and UndefinedBehaviorSanitizer (every UB report
    fatal) for checking the oracle's own memory accesses and arithmetic on the CPU."""
    out = _LIB_SAN if sanitize else _LIB_DEFAULT
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"] \
            if sanitize else []
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra", *san,
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        c_long, c_int, c_double = ctypes.c_long, ctypes.c_int, ctypes.c_double
        L.orc_conv2d.argtypes = [_D, c_long, c_long, _D, c_int, c_int, c_double, _D, c_int]
        L.orc_conv2d_pts.argtypes = [_D, c_long, c_long, _D, c_int, c_int, c_double, _L, _L, c_long, _D, c_int]
        L.orc_conv_sep.argtypes = [_D, c_long, c_long, _D, _D, c_int, c_int, c_double, _D, _D, c_int]
        L.orc_conv_sep_pts.argtypes = [_D, c_long, c_long, _D, _D, c_int, c_int, c_double, _L, _L, c_long, _D,
                                       c_int]
        L.orc_conv3d_sep.argtypes = [_D, c_long, c_long, c_long, _D, _D, _D, c_int, c_int, c_double, _D, c_int]
        L.orc_conv3d_sep_pts.argtypes = [_D, c_long, c_long, c_long, _D, _D, _D, c_int, c_int, c_double, _L, _L, _L,
                                         c_long, _D, c_int]
        L.orc_conv2d_u8.argtypes = [_U8, c_long, c_long, _I16, c_int, c_int, c_int, c_int, _U8, c_int]
        L.orc_conv2d_u8_pts.argtypes = [_U8, c_long, c_long, _I16, c_int, c_int, c_int, c_int, _L, _L, c_long,
                                        _U8, c_int]
        L.orc_harris.argtypes = [_D, c_long, c_long, _D, c_int, c_double, _D, _D, _D, _D, _D, c_int]
        L.orc_harris_pts.argtypes = [_D, c_long, c_long, _D, c_int, c_double, _L, _L, c_long,
                                     _D, _D, _D, _D, c_int]
        L.orc_harris_scale_pts.argtypes = [_D, c_long, c_long, _D, c_int, c_double, _L, _L, c_long, _D, c_int]
        L.orc_harris_f32_bound_pts.argtypes = [_D, c_long, c_long, _D, c_int, c_double, _L, _L, c_long, _D,
                                               c_int]
        L.orc_nms.argtypes = [_D, c_long, c_long, c_int, c_double, _U8, c_int]
        L.orc_bank_fwd.argtypes = [_D, _D, c_long, c_long, c_long, c_long, c_int, _D, c_int]
        L.orc_sse_loss.argtypes = [_D, _D, c_long, _D]
        L.orc_sse_loss.restype = c_double
        L.orc_bank_bwd_input.argtypes = [_D, _D, c_long, c_long, c_long, c_long, c_int, _D, c_int]
        L.orc_bank_bwd_input_pts.argtypes = [_D, _D, c_long, c_long, c_long, c_long, c_int,
                                             _L, _L, _L, c_long, _D, c_int]
        L.orc_bank_bwd_filter.argtypes = [_D, _D, c_long, c_long, c_long, c_long, c_int,
                                          c_long, c_long, _D, c_int]
        L.orc_decode_f16.argtypes = [_U16, _D, c_long]
        L.orc_decode_bf16.argtypes = [_U16, _D, c_long]
        L.orc_encode_f16.argtypes = [_D, _U16, c_long]
        L.orc_encode_bf16.argtypes = [_D, _U16, c_long]
        _lib = L
    return _lib


def _threads(nthreads):
    return int(nthreads) if nthreads else (os.cpu_count() or 1)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_D):
    return a.ctypes.data_as(t)


def _pts(xs, ys):
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    assert xs.shape == ys.shape
    return xs, ys


# ----------------------------------------------------------------------------- storage codecs

def decode(bits_or_values: np.ndarray, dtype: str) -> np.ndarray:
    """Stored pixels -> float64.  dtype in {'f32', 'f16', 'bf16', 'u8', 'f64'}; f16/bf16 take uint16 bits."""
    a = np.asarray(bits_or_values)
    if dtype in ("f32", "u8", "f64"):
        return a.astype(np.float64)
    bits = np.ascontiguousarray(a, dtype=np.uint16)
    out = np.empty(bits.shape, dtype=np.float64)
    fn = lib().orc_decode_f16 if dtype == "f16" else lib().orc_decode_bf16
    fn(_p(bits, _U16), _p(out), bits.size)
    return out


def encode(values: np.ndarray, dtype: str) -> np.ndarray:
    """float64 -> binary16 / bfloat16 bits, round to nearest even."""
    v = _f64(values)
    out = np.empty(v.shape, dtype=np.uint16)
    fn = lib().orc_encode_f16 if dtype == "f16" else lib().orc_encode_bf16
    fn(_p(v), _p(out, _U16), v.size)
    return out


# ----------------------------------------------------------------------------- stencils
# border: "clamp" (closest pixel inside, Fig. 3a) or "constant" (reads outside return
# `constant`, Fig. 3b).

def conv2d(X, w, nthreads=None, border="clamp", constant=0.0):
    X = _f64(X)
    w = _f64(w)
    H, W = X.shape
    r = (w.shape[-1] - 1) // 2
    assert w.size == (2 * r + 1) ** 2
    Y = np.empty_like(X)
    lib().orc_conv2d(_p(X), W, H, _p(w), r, BORDERS[border], float(constant), _p(Y), _threads(nthreads))
    return Y


def conv2d_pts(X, w, xs, ys, nthreads=None, border="clamp", constant=0.0):
    X = _f64(X)
    w = _f64(w)
    H, W = X.shape
    r = (w.shape[-1] - 1) // 2
    xs, ys = _pts(xs, ys)
    out = np.empty(xs.shape, dtype=np.float64)
    lib().orc_conv2d_pts(_p(X), W, H, _p(w), r, BORDERS[border], float(constant), _p(xs, _L), _p(ys, _L),
                         xs.size, _p(out), _threads(nthreads))
    return out


def conv_sep(X, h, v, nthreads=None, return_intermediate=False, border="clamp", constant=0.0):
    X = _f64(X)
    h = _f64(h)
    v = _f64(v)
    H, W = X.shape
    r = (h.size - 1) // 2
    assert h.size == v.size == 2 * r + 1
    T = np.empty_like(X)
    Y = np.empty_like(X)
    lib().orc_conv_sep(_p(X), W, H, _p(h), _p(v), r, BORDERS[border], float(constant), _p(T), _p(Y),
                       _threads(nthreads))
    return (Y, T) if return_intermediate else Y


def conv_sep_pts(X, h, v, xs, ys, nthreads=None, border="clamp", constant=0.0):
    X = _f64(X)
    h = _f64(h)
    v = _f64(v)
    H, W = X.shape
    r = (h.size - 1) // 2
    xs, ys = _pts(xs, ys)
    out = np.empty(xs.shape, dtype=np.float64)
    lib().orc_conv_sep_pts(_p(X), W, H, _p(h), _p(v), r, BORDERS[border], float(constant), _p(xs, _L),
                           _p(ys, _L), xs.size, _p(out), _threads(nthreads))
    return out


def conv3d_sep(X, hx, hy, hz, nthreads=None, border="clamp", constant=0.0):
    """X [D, H, W] (slice, row, column): separable 3-D correlation through the boundary."""
    X = _f64(X)
    hx, hy, hz = _f64(hx), _f64(hy), _f64(hz)
    D, H, W = X.shape
    r = (hx.size - 1) // 2
    assert hx.size == hy.size == hz.size == 2 * r + 1
    Y = np.empty_like(X)
    lib().orc_conv3d_sep(_p(X), W, H, D, _p(hx), _p(hy), _p(hz), r, BORDERS[border], float(constant), _p(Y),
                         _threads(nthreads))
    return Y


def conv3d_sep_pts(X, hx, hy, hz, xs, ys, zs, nthreads=None, border="clamp", constant=0.0):
    X = _f64(X)
    hx, hy, hz = _f64(hx), _f64(hy), _f64(hz)
    D, H, W = X.shape
    r = (hx.size - 1) // 2
    xs, ys = _pts(xs, ys)
    zs = np.ascontiguousarray(zs, dtype=np.int64)
    out = np.empty(xs.shape, dtype=np.float64)
    lib().orc_conv3d_sep_pts(_p(X), W, H, D, _p(hx), _p(hy), _p(hz), r, BORDERS[border], float(constant),
                             _p(xs, _L), _p(ys, _L), _p(zs, _L), xs.size, _p(out), _threads(nthreads))
    return out


def normwise_scale_sep3d(X, hx, hy, hz, nthreads=None, border="clamp", constant=0.0):
    return conv3d_sep(np.abs(_f64(X)), np.abs(_f64(hx)), np.abs(_f64(hy)), np.abs(_f64(hz)), nthreads,
                      border=border, constant=abs(constant))


def _u8_args(X, w, shift, constant):
    X = np.ascontiguousarray(X, dtype=np.uint8)
    w = np.ascontiguousarray(w, dtype=np.int16)
    r = (w.shape[-1] - 1) // 2
    assert w.size == (2 * r + 1) ** 2
    assert 0 <= int(shift) <= 16 and 0 <= int(constant) <= 255
    return X, w, r


def conv2d_u8(X, w, shift, nthreads=None, border="clamp", constant=0):
    """Integer correlation of an unsigned char image: exact sum, round (ties up), saturate."""
    X, w, r = _u8_args(X, w, shift, constant)
    H, W = X.shape
    Y = np.empty_like(X)
    lib().orc_conv2d_u8(_p(X, _U8), W, H, _p(w, _I16), r, int(shift), BORDERS[border], int(constant),
                        _p(Y, _U8), _threads(nthreads))
    return Y


def conv2d_u8_pts(X, w, shift, xs, ys, nthreads=None, border="clamp", constant=0):
    X, w, r = _u8_args(X, w, shift, constant)
    H, W = X.shape
    xs, ys = _pts(xs, ys)
    out = np.empty(xs.shape, dtype=np.uint8)
    lib().orc_conv2d_u8_pts(_p(X, _U8), W, H, _p(w, _I16), r, int(shift), BORDERS[border], int(constant),
                            _p(xs, _L), _p(ys, _L), xs.size, _p(out, _U8), _threads(nthreads))
    return out


def harris(X, g, k, nthreads=None, windows=False):
    """R (and optionally Sxx, Syy, Sxy) for the whole image."""
    X = _f64(X)
    g = _f64(g)
    H, W = X.shape
    rg = (g.size - 1) // 2
    R = np.empty_like(X)
    S = [np.empty_like(X) for _ in range(3)] if windows else [None, None, None]
    work = np.empty(5 * X.size, dtype=np.float64)
    nul = ctypes.cast(None, _D)
    lib().orc_harris(_p(X), W, H, _p(g), rg, float(k), _p(R),
                     *[(_p(s) if s is not None else nul) for s in S], _p(work), _threads(nthreads))
    return (R, *S) if windows else R


def harris_pts(X, g, k, xs, ys, nthreads=None):
    """(R, Sxx, Syy, Sxy) at the given pixels."""
    X = _f64(X)
    g = _f64(g)
    H, W = X.shape
    rg = (g.size - 1) // 2
    xs, ys = _pts(xs, ys)
    outs = [np.empty(xs.shape, dtype=np.float64) for _ in range(4)]
    lib().orc_harris_pts(_p(X), W, H, _p(g), rg, float(k), _p(xs, _L), _p(ys, _L), xs.size,
                         *[_p(o) for o in outs], _threads(nthreads))
    return tuple(outs)


def harris_scale_pts(X, g, k, xs, ys, nthreads=None):
    """Normwise scale of the response at the given pixels (absolute-value evaluation; see the C source)."""
    X = _f64(X)
    g = _f64(g)
    H, W = X.shape
    rg = (g.size - 1) // 2
    xs, ys = _pts(xs, ys)
    out = np.empty(xs.shape, dtype=np.float64)
    lib().orc_harris_scale_pts(_p(X), W, H, _p(g), rg, float(k), _p(xs, _L), _p(ys, _L), xs.size, _p(out),
                               _threads(nthreads))
    return out


def harris_scale(X, g, k, nthreads=None):
    """harris_scale_pts at every pixel, as an H x W array."""
    H, W = np.shape(X)
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return harris_scale_pts(X, g, k, xs.ravel(), ys.ravel(), nthreads).reshape(H, W)


def harris_f32_bound_pts(X, g, k, xs, ys, nthreads=None):
    """Bound on |R_float32 - R| at the given pixels for any float32 evaluation order of the
    Harris chain (Sobel, products, window, response); see the C source for the derivation."""
    X = _f64(X)
    g = _f64(g)
    H, W = X.shape
    rg = (g.size - 1) // 2
    xs, ys = _pts(xs, ys)
    out = np.empty(xs.shape, dtype=np.float64)
    lib().orc_harris_f32_bound_pts(_p(X), W, H, _p(g), rg, float(k), _p(xs, _L), _p(ys, _L), xs.size, _p(out),
                                   _threads(nthreads))
    return out


def harris_f32_bound(X, g, k, nthreads=None):
    """harris_f32_bound_pts at every pixel, as an H x W array."""
    H, W = np.shape(X)
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return harris_f32_bound_pts(X, g, k, xs.ravel(), ys.ravel(), nthreads).reshape(H, W)


def nms(R, tau, radius=1, nthreads=None):
    R = _f64(R)
    H, W = R.shape
    M = np.empty((H, W), dtype=np.uint8)
    lib().orc_nms(_p(R), W, H, int(radius), float(tau), _p(M, _U8), _threads(nthreads))
    return M


# ----------------------------------------------------------------------------- filter bank

def bank_fwd(x, w, nthreads=None):
    """x [N,1,H,W] or [N,H,W], w [F,k,k] -> y [N,F,H,W]."""
    x = _f64(x)
    w = _f64(w)
    N, H, W = x.shape[0], x.shape[-2], x.shape[-1]
    F = w.shape[0]
    r = (w.shape[-1] - 1) // 2
    y = np.empty((N, F, H, W), dtype=np.float64)
    lib().orc_bank_fwd(_p(x), _p(w), N, F, H, W, r, _p(y), _threads(nthreads))
    return y


def sse_loss(y, t, want_grad=True):
    y = _f64(y)
    t = _f64(t)
    gy = np.empty_like(y) if want_grad else None
    L = lib().orc_sse_loss(_p(y), _p(t), y.size, _p(gy) if want_grad else ctypes.cast(None, _D))
    return (L, gy) if want_grad else L


def bank_bwd_input(gy, w, nthreads=None):
    gy = _f64(gy)
    w = _f64(w)
    N, F, H, W = gy.shape
    r = (w.shape[-1] - 1) // 2
    gx = np.empty((N, 1, H, W), dtype=np.float64)
    lib().orc_bank_bwd_input(_p(gy), _p(w), N, F, H, W, r, _p(gx), _threads(nthreads))
    return gx


def bank_bwd_input_pts(gy, w, ns, xs, ys, nthreads=None):
    gy = _f64(gy)
    w = _f64(w)
    N, F, H, W = gy.shape
    r = (w.shape[-1] - 1) // 2
    ns = np.ascontiguousarray(ns, dtype=np.int64)
    xs, ys = _pts(xs, ys)
    out = np.empty(xs.shape, dtype=np.float64)
    lib().orc_bank_bwd_input_pts(_p(gy), _p(w), N, F, H, W, r, _p(ns, _L), _p(xs, _L), _p(ys, _L),
                                 xs.size, _p(out), _threads(nthreads))
    return out


def bank_bwd_filter(gy, x, radius, fk_range=None, nthreads=None):
    """gw [F, 2r+1, 2r+1] (or the flattened taps fk_range=(lo, hi) only)."""
    gy = _f64(gy)
    x = _f64(x)
    N, F, H, W = gy.shape
    nk = (2 * radius + 1) ** 2
    lo, hi = fk_range if fk_range is not None else (0, F * nk)
    gw = np.empty(hi - lo, dtype=np.float64)
    lib().orc_bank_bwd_filter(_p(gy), _p(x), N, F, H, W, int(radius), lo, hi, _p(gw), _threads(nthreads))
    if fk_range is None:
        return gw.reshape(F, 2 * radius + 1, 2 * radius + 1)
    return gw


# ----------------------------------------------------------------------------- tolerance helpers

def normwise_scale_conv2d(X, w, nthreads=None, border="clamp", constant=0.0):
    """S(p) = sum_k |w_k| |X(p+k)|: the same stencil on absolute values."""
    return conv2d(np.abs(_f64(X)), np.abs(_f64(w)), nthreads, border=border, constant=abs(constant))


def normwise_scale_sep(X, h, v, nthreads=None, border="clamp", constant=0.0):
    return conv_sep(np.abs(_f64(X)), np.abs(_f64(h)), np.abs(_f64(v)), nthreads, border=border,
                    constant=abs(constant))


def response_scale(sxx, syy, sxy, k):
    """|Sxx Syy| + Sxy^2 + k (Sxx + Syy)^2: the magnitude the response's rounding error scales with."""
    return np.abs(sxx * syy) + sxy * sxy + abs(k) * (sxx + syy) ** 2
