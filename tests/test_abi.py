"""C-ABI library: loads, exports every declared symbol, and validates arguments on the host.

These tests make no compute call: argument checks run before any device query,
so each error path returns its status code on a machine without a GPU.  The
addresses are fake, so a call here must never pass validation where a GPU is
visible (it would launch on them): every call either fails a check or is an
empty no-op, except in test_no_device_or_launch_path, which is skipped when a
GPU is present.
"""
import ctypes
import os
import re

import pytest

from paper_1605_06399_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "icl.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(icl_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libicl.so is not built (run __graft_entry__.build())")
    return B.lib()


@pytest.fixture
def no_gpu(L):
    """The fake-address validation tests run only where no GPU is visible: should a check
    regress there, the call fails with ICL_ERR_NO_DEVICE instead of launching on fake memory."""
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("fake device addresses are only passed where no GPU is visible")
    return L


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), f"{n} declared in icl.h but not exported"
    assert set(names) == set(B.EXPORTED)


def test_status_strings_and_version(L):
    for s in range(0, 11):
        assert B.status_string(s)
    assert "gfx950" in B.icl_version()


def test_variant_tables(L):
    for op in range(B.ICL_OP_COUNT):
        n = B.icl_variant_count(op)
        assert n >= 1
        names = B.variant_names(op)
        assert all(names) and len(set(names)) == n
        assert B.icl_variant_name(op, n) is None
    assert B.variant_names(B.ICL_OP_CONV_SEP)[0] == "plain2p"
    assert B.variant_names(B.ICL_OP_CONV2D)[0] == "plain"
    assert B.icl_force_variant(B.ICL_OP_CONV2D, 99) == B.ICL_ERR_INVALID_VALUE
    assert B.icl_force_variant(B.ICL_OP_COUNT, 0) == B.ICL_ERR_INVALID_VALUE


def test_workspace_sizes(L):
    st, nb = B.icl_workspace_size(B.ICL_OP_CONV_SEP, 100, 7)
    assert st == B.ICL_OK and nb == 100 * 7 * 4
    st, nb = B.icl_workspace_size(B.ICL_OP_HARRIS, 10, 10)
    assert st == B.ICL_OK and nb == 2 * 100 * 4
    st, nb = B.icl_workspace_size(B.ICL_OP_CONV2D, 10, 10)
    assert st == B.ICL_OK and nb == 0
    st, nb = B.icl_workspace_size(B.ICL_OP_BANK_BWD_FILTER, 1024, 1024, 32, 16, 4)
    assert st == B.ICL_OK and nb == 32 * 32 * 16 * 16 * 81 * 4
    assert B.icl_workspace_size(B.ICL_OP_BANK_BWD_FILTER, 8, 8, 1, 1, 9)[0] == B.ICL_ERR_RADIUS
    assert B.icl_workspace_size(B.ICL_OP_CONV_SEP, -1, 7)[0] == B.ICL_ERR_INVALID_VALUE
    assert B.icl_workspace_size(B.ICL_OP_CONV_SEP, 1, 7, dtype=7)[0] == B.ICL_ERR_DTYPE
    assert B.icl_workspace_size(42, 1, 7)[0] == B.ICL_ERR_INVALID_VALUE
    st, nb = B.icl_workspace_size(B.ICL_OP_CONV2D_U8, 10, 10, dtype=B.ICL_U8)
    assert st == B.ICL_OK and nb == 0
    assert B.icl_workspace_size(B.ICL_OP_CONV2D_U8, 10, 10, dtype=B.ICL_F32)[0] == B.ICL_ERR_DTYPE
    assert B.icl_workspace_size(B.ICL_OP_CONV_SEP, 10, 10, dtype=B.ICL_U8)[0] == B.ICL_ERR_DTYPE


# Fake "device" addresses: never dereferenced, because validation fails (or the
# device check does) before anything is launched.
SRC, DST, TAPS, WS = 0x10000000, 0x20000000, 0x30000000, 0x40000000


def sep(**kw):
    a = dict(src=SRC, src_pitch=64 * 4, dst=DST, dst_pitch=64 * 4, width=64, height=8, dtype=B.ICL_F32,
             taps_x=TAPS, taps_y=TAPS, radius=2, workspace=0, workspace_bytes=0)
    a.update(kw)
    return B.icl_conv_sep(*a.values())


def test_conv_sep_validation(no_gpu):
    assert sep(width=-1) == B.ICL_ERR_INVALID_VALUE
    assert sep(height=-3) == B.ICL_ERR_INVALID_VALUE
    assert sep(dtype=5) == B.ICL_ERR_DTYPE
    assert sep(radius=-1) == B.ICL_ERR_RADIUS
    assert sep(radius=B.ICL_MAX_RADIUS + 1) == B.ICL_ERR_RADIUS
    assert sep(width=0) == B.ICL_OK                              # empty image: no-op
    assert sep(height=0, src=0, dst=0) == B.ICL_OK
    assert sep(src=0) == B.ICL_ERR_INVALID_VALUE
    assert sep(taps_y=0) == B.ICL_ERR_INVALID_VALUE
    assert sep(src_pitch=63 * 4) == B.ICL_ERR_PITCH
    assert sep(dst_pitch=64 * 4 + 1) == B.ICL_ERR_PITCH
    assert sep(dtype=B.ICL_F16, src_pitch=129, dst_pitch=128) == B.ICL_ERR_PITCH
    assert sep(dst=SRC + 7 * 256) == B.ICL_ERR_ALIAS              # last source row overlaps
    assert sep(workspace=DST + 100, workspace_bytes=4096) == B.ICL_ERR_ALIAS


def test_conv2d_harris_nms_validation(no_gpu):
    assert B.icl_conv2d(SRC, 256, DST, 256, 64, 8, B.ICL_F32, TAPS, 17) == B.ICL_ERR_RADIUS
    assert B.icl_conv2d(SRC, 256, DST, 256, 64, 8, B.ICL_F32, 0, 1) == B.ICL_ERR_INVALID_VALUE
    assert B.icl_conv2d(SRC, 256, SRC, 256, 64, 8, B.ICL_F32, TAPS, 1) == B.ICL_ERR_ALIAS
    assert B.icl_conv2d(SRC, 256, DST, 256, 0, 8, B.ICL_F32, TAPS, 1) == B.ICL_OK
    assert B.icl_harris(SRC, 256, DST, 256, 64, 8, TAPS, 8, 0.04) == B.ICL_ERR_RADIUS
    assert B.icl_harris(SRC, 100, DST, 256, 64, 8, TAPS, 2, 0.04) == B.ICL_ERR_PITCH
    assert B.icl_harris(SRC, 256, SRC + 4, 256, 64, 8, TAPS, 2, 0.04) == B.ICL_ERR_ALIAS
    assert B.icl_nms(SRC, 256, DST, 64, 64, 8, 0, 1e-3) == B.ICL_ERR_RADIUS
    assert B.icl_nms(SRC, 256, DST, 63, 64, 8, 1, 1e-3) == B.ICL_ERR_PITCH
    assert B.icl_nms(SRC, 256, SRC + 64, 64, 64, 8, 1, 1e-3) == B.ICL_ERR_ALIAS
    assert B.icl_nms(SRC, 256, DST, 64, -1, 8, 1, 1e-3) == B.ICL_ERR_INVALID_VALUE


def test_border_and_u8_validation(no_gpu):
    C, K = B.ICL_BORDER_CLAMP, B.ICL_BORDER_CONSTANT
    sb = B.icl_conv_sep_border
    assert sb(SRC, 256, DST, 256, 64, 8, B.ICL_F32, TAPS, TAPS, 2, 2, 0.0) == B.ICL_ERR_INVALID_VALUE
    assert sb(SRC, 256, DST, 256, 64, 8, B.ICL_F32, TAPS, TAPS, 2, -1, 0.0) == B.ICL_ERR_INVALID_VALUE
    assert sb(SRC, 256, DST, 256, 64, 8, B.ICL_U8, TAPS, TAPS, 2, K, 0.0) == B.ICL_ERR_DTYPE
    assert sb(SRC, 256, DST, 256, 64, 8, B.ICL_F32, TAPS, TAPS, 17, K, 0.0) == B.ICL_ERR_RADIUS
    assert sb(SRC, 256, SRC + 4, 256, 64, 8, B.ICL_F32, TAPS, TAPS, 2, K, 0.5) == B.ICL_ERR_ALIAS
    assert sb(SRC, 256, DST, 256, 0, 8, B.ICL_F32, TAPS, TAPS, 2, K, 0.5) == B.ICL_OK
    c2 = B.icl_conv2d_border
    assert c2(SRC, 256, DST, 256, 64, 8, B.ICL_F32, TAPS, 2, 5, 0.0) == B.ICL_ERR_INVALID_VALUE
    assert c2(SRC, 256, DST, 256, 64, 8, B.ICL_U8, TAPS, 2, C, 0.0) == B.ICL_ERR_DTYPE
    assert c2(SRC, 256, DST, 256, 64, 8, B.ICL_F32, 0, 2, K, 1.0) == B.ICL_ERR_INVALID_VALUE
    assert c2(SRC, 255, DST, 256, 64, 8, B.ICL_F32, TAPS, 2, K, 1.0) == B.ICL_ERR_PITCH
    assert c2(SRC, 256, DST, 256, 64, 0, B.ICL_F32, TAPS, 2, K, 1.0) == B.ICL_OK
    u8 = B.icl_conv2d_u8
    assert u8(SRC, 64, DST, 64, 64, 8, TAPS, 8, 12) == B.ICL_ERR_RADIUS
    assert u8(SRC, 64, DST, 64, 64, 8, TAPS, -1, 12) == B.ICL_ERR_RADIUS
    assert u8(SRC, 64, DST, 64, 64, 8, TAPS, 2, 17) == B.ICL_ERR_INVALID_VALUE
    assert u8(SRC, 64, DST, 64, 64, 8, TAPS, 2, -1) == B.ICL_ERR_INVALID_VALUE
    assert u8(SRC, 64, DST, 64, 64, 8, TAPS, 2, 12, 3, 0) == B.ICL_ERR_INVALID_VALUE
    assert u8(SRC, 64, DST, 64, 64, 8, TAPS, 2, 12, K, 256) == B.ICL_ERR_INVALID_VALUE
    assert u8(SRC, 64, DST, 64, 64, 8, TAPS, 2, 12, K, -1) == B.ICL_ERR_INVALID_VALUE
    assert u8(SRC, 63, DST, 64, 64, 8, TAPS, 2, 12) == B.ICL_ERR_PITCH
    assert u8(0, 64, DST, 64, 64, 8, TAPS, 2, 12) == B.ICL_ERR_INVALID_VALUE
    assert u8(SRC, 64, DST, 64, 64, 8, 0, 2, 12) == B.ICL_ERR_INVALID_VALUE
    assert u8(SRC, 64, SRC + 7 * 64, 64, 64, 8, TAPS, 2, 12) == B.ICL_ERR_ALIAS
    assert u8(SRC, 64, DST, 64, -1, 8, TAPS, 2, 12) == B.ICL_ERR_INVALID_VALUE
    assert u8(SRC, 64, DST, 64, 0, 8, TAPS, 2, 12) == B.ICL_OK


def test_corners_validation(no_gpu):
    c = B.icl_corners
    MASK, RESP = 0x50000000, 0x60000000
    assert c(SRC, 256, MASK, 64, 64, 8, TAPS, 8, 0.04, 1, 1e-3) == B.ICL_ERR_RADIUS
    assert c(SRC, 256, MASK, 64, 64, 8, TAPS, 2, 0.04, 0, 1e-3) == B.ICL_ERR_RADIUS
    assert c(SRC, 256, MASK, 64, 64, 8, TAPS, 2, 0.04, 8, 1e-3) == B.ICL_ERR_RADIUS
    assert c(SRC, 255, MASK, 64, 64, 8, TAPS, 2, 0.04, 1, 1e-3) == B.ICL_ERR_PITCH
    assert c(SRC, 256, MASK, 63, 64, 8, TAPS, 2, 0.04, 1, 1e-3) == B.ICL_ERR_PITCH
    assert c(SRC, 256, MASK, 64, 64, 8, TAPS, 2, 0.04, 1, 1e-3, RESP, 100) == B.ICL_ERR_PITCH
    assert c(SRC, 256, MASK, 64, 64, 8, 0, 2, 0.04, 1, 1e-3) == B.ICL_ERR_INVALID_VALUE
    assert c(SRC, 256, SRC + 100, 64, 64, 8, TAPS, 2, 0.04, 1, 1e-3) == B.ICL_ERR_ALIAS
    assert c(SRC, 256, MASK, 64, 64, 8, TAPS, 2, 0.04, 1, 1e-3, SRC + 256, 256) == B.ICL_ERR_ALIAS
    assert c(SRC, 256, MASK, 64, 64, 8, TAPS, 2, 0.04, 1, 1e-3, MASK + 8, 256) == B.ICL_ERR_ALIAS
    assert c(SRC, 256, MASK, 64, 64, 8, TAPS, 2, 0.04, 1, 1e-3, 0, 0, MASK + 4, 64) == B.ICL_ERR_ALIAS
    assert c(SRC, 256, MASK, 64, -1, 8, TAPS, 2, 0.04, 1, 1e-3) == B.ICL_ERR_INVALID_VALUE
    assert c(SRC, 256, MASK, 64, 0, 8, TAPS, 2, 0.04, 1, 1e-3) == B.ICL_OK


def test_conv3d_validation(no_gpu):
    def c3(**kw):
        a = dict(src=SRC, srp=256, ssp=256 * 8, dst=DST, drp=256, dsp=256 * 8, w=64, h=8, d=4, dt=B.ICL_F32,
                 tx=TAPS, ty=TAPS, tz=TAPS, r=2, border=B.ICL_BORDER_CLAMP, c=0.0, ws=0, wsb=0)
        a.update(kw)
        return B.icl_conv3d_sep(*a.values())
    assert c3(d=-1) == B.ICL_ERR_INVALID_VALUE
    assert c3(r=8) == B.ICL_ERR_RADIUS
    assert c3(dt=B.ICL_U8) == B.ICL_ERR_DTYPE
    assert c3(border=4) == B.ICL_ERR_INVALID_VALUE
    assert c3(srp=255) == B.ICL_ERR_PITCH
    assert c3(ssp=256 * 7) == B.ICL_ERR_PITCH
    assert c3(dsp=256 * 8 + 2) == B.ICL_ERR_PITCH
    assert c3(tz=0) == B.ICL_ERR_INVALID_VALUE
    assert c3(dst=SRC + 256 * 8 * 3) == B.ICL_ERR_ALIAS
    assert c3(ws=DST + 64, wsb=1024) == B.ICL_ERR_ALIAS
    assert c3(d=0) == B.ICL_OK
    st, nb = B.icl_workspace_size(B.ICL_OP_CONV3D_SEP, 10, 20, n=30)
    assert st == B.ICL_OK and nb == 2 * 10 * 20 * 30 * 4


def test_bank_and_loss_validation(no_gpu):
    assert B.icl_bank_fwd(SRC, TAPS, DST, 2, 16, 8, 8, 5) == B.ICL_ERR_RADIUS
    assert B.icl_bank_fwd(SRC, TAPS, DST, 2, 0, 8, 8, 4) == B.ICL_ERR_INVALID_VALUE
    assert B.icl_bank_fwd(SRC, TAPS, DST, 2, 65, 8, 8, 4) == B.ICL_ERR_UNSUPPORTED
    assert B.icl_bank_fwd(SRC, TAPS, SRC + 4, 2, 4, 8, 8, 4) == B.ICL_ERR_ALIAS
    assert B.icl_bank_fwd(SRC, TAPS, DST, 0, 4, 8, 8, 4) == B.ICL_OK
    assert B.icl_bank_bwd_input(0, TAPS, DST, 2, 4, 8, 8, 4) == B.ICL_ERR_INVALID_VALUE
    assert B.icl_bank_bwd_filter(SRC, DST, WS, 2, 4, 8, 8, 4, 0, 0) == B.ICL_ERR_WORKSPACE
    assert B.icl_bank_bwd_filter(SRC, DST, WS, 2, 4, 8, 8, 4, 0x50000000, 10) == B.ICL_ERR_WORKSPACE
    # fused forward + loss: x 512 B, y / gy / t 2 KiB each at these sizes
    TG, GY, LS = 0x50000000, 0x60000000, 0x70000000
    _, wsb = B.icl_workspace_size(B.ICL_OP_BANK_FWD_SSE, 8, 8, 2, 4, 4)
    assert wsb >= 8

    def fs(**kw):
        a = dict(x=SRC, w=TAPS, t=TG, y=0, gy=GY, loss=LS, n=2, f=4, h=8, wd=8, r=4, ws=WS, wsb=wsb)
        a.update(kw)
        return B.icl_bank_fwd_sse(*a.values())
    assert fs(r=5) == B.ICL_ERR_RADIUS
    assert fs(f=65) == B.ICL_ERR_UNSUPPORTED
    assert fs(loss=0) == B.ICL_ERR_INVALID_VALUE
    assert fs(t=0) == B.ICL_ERR_INVALID_VALUE
    assert fs(ws=0) == B.ICL_ERR_WORKSPACE
    assert fs(wsb=wsb - 1) == B.ICL_ERR_WORKSPACE
    assert fs(gy=SRC + 4) == B.ICL_ERR_ALIAS          # gradient over x
    assert fs(y=GY + 1024) == B.ICL_ERR_ALIAS         # y over gy
    assert fs(y=TG) == B.ICL_ERR_ALIAS                # y over the target
    assert fs(loss=TG + 2044) == B.ICL_ERR_ALIAS      # loss scalar inside the target
    assert fs(ws=GY + 8) == B.ICL_ERR_ALIAS           # workspace over gy
    assert B.icl_sse_loss(SRC, DST, 0, -1, WS) == B.ICL_ERR_INVALID_VALUE
    assert B.icl_sse_loss(SRC, DST, 0, 10, WS, 0, 0) == B.ICL_ERR_WORKSPACE
    assert B.icl_sse_loss(SRC, DST, SRC + 8, 10, WS, 0x50000000, 1 << 20) == B.ICL_ERR_ALIAS


def test_batch_plan_validation(no_gpu):
    d = B.icl_image_desc(SRC, DST, 256, 256, 64, 8, 3, TAPS, TAPS)
    assert B.icl_batch_plan_create([d], 9)[0] == B.ICL_ERR_DTYPE
    bad = B.icl_image_desc(SRC, DST, 256, 256, 64, 8, 8, TAPS, TAPS)
    assert B.icl_batch_plan_create([bad], B.ICL_F16)[0] == B.ICL_ERR_RADIUS
    bad = B.icl_image_desc(SRC, DST, 100, 256, 64, 8, 1, TAPS, TAPS)
    assert B.icl_batch_plan_create([bad], B.ICL_F16)[0] == B.ICL_ERR_PITCH
    bad = B.icl_image_desc(SRC, SRC + 256, 256, 256, 64, 8, 1, TAPS, TAPS)
    assert B.icl_batch_plan_create([bad], B.ICL_F32)[0] == B.ICL_ERR_ALIAS
    d2 = B.icl_image_desc(SRC + (1 << 20), DST + 1024, 256, 256, 64, 8, 1, TAPS, TAPS)   # outputs overlap
    assert B.icl_batch_plan_create([d, d2], B.ICL_F32)[0] == B.ICL_ERR_ALIAS
    d3 = B.icl_image_desc(DST + 512, DST + (1 << 20), 256, 256, 64, 8, 1, TAPS, TAPS)    # input of 3 = output of 1
    assert B.icl_batch_plan_create([d, d3], B.ICL_F32)[0] == B.ICL_ERR_ALIAS
    assert B.lib().icl_conv_sep_batched(None, None) == B.ICL_ERR_INVALID_VALUE


def test_no_device_or_launch_path(L):
    """A valid call either reports that no GPU is visible or succeeds (a GPU is present)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present: compute calls are covered by the gpu tests")
    assert B.icl_init() == B.ICL_ERR_NO_DEVICE
    assert sep() == B.ICL_ERR_NO_DEVICE
    assert sep(dst=SRC + 8 * 256) == B.ICL_ERR_NO_DEVICE         # adjacent rows are no alias
    assert B.icl_conv2d_u8(SRC, 64, SRC + 8 * 64, 64, 64, 8, TAPS, 2, 12, B.ICL_BORDER_CONSTANT,
                           255) == B.ICL_ERR_NO_DEVICE
    assert B.icl_conv_sep_border(SRC, 256, DST, 256, 64, 8, B.ICL_F32, TAPS, TAPS, 2, B.ICL_BORDER_CONSTANT,
                                 0.5) == B.ICL_ERR_NO_DEVICE
    _, wsb = B.icl_workspace_size(B.ICL_OP_BANK_FWD_SSE, 8, 8, 2, 4, 4)
    # loss scalar right after the target, y absent: valid, so it reaches the device check
    assert B.icl_bank_fwd_sse(SRC, TAPS, 0x50000000, 0, 0x60000000, 0x50000000 + 2048, 2, 4, 8, 8, 4,
                              WS, wsb) == B.ICL_ERR_NO_DEVICE
    assert B.icl_tune(B.ICL_OP_CONV_SEP, B.ICL_F32, 2, 64, 64) == B.ICL_ERR_NO_DEVICE


def test_perf_model_learns_a_smooth_function(L):
    """The tuner's time model is host code: it must fit a smooth function of a few features
    well enough to rank unseen points, deterministically."""
    import numpy as np
    rng = np.random.default_rng(7)
    f = lambda X: 1.5 * X[:, 0] - 2.0 * X[:, 1] + 0.5 * X[:, 0] * X[:, 2] + 3.0   # noqa: E731
    X = rng.uniform(-1, 1, (48, 3))
    Xq = rng.uniform(-1, 1, (24, 3))
    st, yq = B.icl_perf_model_fit_predict(X, f(X), Xq, hidden=8, iters=3000, seed=11)
    assert st == B.ICL_OK
    resid = yq - f(Xq)
    r2 = 1.0 - np.sum(resid ** 2) / np.sum((f(Xq) - f(Xq).mean()) ** 2)
    assert r2 > 0.95, r2
    # ranking: the predicted best of the held-out points is among the true best three
    assert np.argmin(yq) in np.argsort(f(Xq))[:3]
    st2, yq2 = B.icl_perf_model_fit_predict(X, f(X), Xq, hidden=8, iters=3000, seed=11)
    assert st2 == B.ICL_OK and np.array_equal(yq, yq2)
    # a constant target is predicted exactly; invalid arguments are refused
    st, yc = B.icl_perf_model_fit_predict(X, np.full(48, 2.5), Xq, seed=1)
    assert st == B.ICL_OK and np.allclose(yc, 2.5, atol=1e-9)
    assert B.icl_perf_model_fit_predict(X[:1], f(X[:1]), Xq)[0] == B.ICL_ERR_INVALID_VALUE
    assert B.icl_perf_model_fit_predict(X, f(X), Xq, hidden=0)[0] == B.ICL_ERR_INVALID_VALUE
    assert B.icl_perf_model_fit_predict(X, f(X), Xq, iters=0)[0] == B.ICL_ERR_INVALID_VALUE


def test_tune_model_validation(no_gpu):
    assert B.icl_tune_model(B.ICL_OP_CONV_SEP, B.ICL_F32, 2, 64, 64, 1, 2)[0] == B.ICL_ERR_INVALID_VALUE
    assert B.icl_tune_model(B.ICL_OP_CONV_SEP, B.ICL_F32, 2, 64, 64, 4, 0)[0] == B.ICL_ERR_INVALID_VALUE
    assert B.icl_tune_model(B.ICL_OP_CONV_SEP, B.ICL_F32, 2, 64, 64, 4, 2)[0] == B.ICL_ERR_NO_DEVICE


def test_tune_cache_file_roundtrip_and_corruption(L, tmp_path):
    p = tmp_path / "cache.json"
    assert B.icl_tune_save(str(p)) == B.ICL_OK
    assert B.icl_tune_load(str(p)) == B.ICL_OK
    p.write_text("{not json")
    assert B.icl_tune_load(str(p)) == B.ICL_ERR_TUNE_CACHE
    assert B.icl_tune_load(str(tmp_path / "missing.json")) == B.ICL_ERR_TUNE_CACHE
    # an entry for another device or an unknown variant never selects a kernel
    p.write_text('{"version": 1, "entries": [\n  {"key": "gfx000|1|conv2d|0|3|20", "variant": "nope", "us": 1.0}\n]}\n')
    assert B.icl_tune_load(str(p)) == B.ICL_OK
    st, idx = B.icl_selected_variant(B.ICL_OP_CONV2D, B.ICL_F32, 3, 1024, 1024)
    assert st == B.ICL_OK and idx == 1      # the default (first LDS variant), not the foreign entry
    B.icl_tune_clear()


def test_math_mode_and_variant_arithmetic(L):
    assert B.icl_get_math() == B.ICL_MATH_F32
    assert B.icl_set_math(2) == B.ICL_ERR_INVALID_VALUE and B.icl_get_math() == B.ICL_MATH_F32
    names = B.variant_names(B.ICL_OP_CONV2D)
    for i, n in enumerate(names):
        want = "fp16x3_mfma" if n.startswith("mfma_f16") else "fp32_valu"
        assert B.icl_variant_arith(B.ICL_OP_CONV2D, i) == want, n
    for op in (B.ICL_OP_BANK_FWD, B.ICL_OP_BANK_BWD_FILTER, B.ICL_OP_BANK_FWD_SSE):
        for i, n in enumerate(B.variant_names(op)):
            assert B.icl_variant_arith(op, i) == ("fp32_mfma" if "mfma" in n else "fp32_valu"), n
    assert all(B.icl_variant_arith(B.ICL_OP_CONV2D_U8, i) == "int32_valu"
               for i in range(B.icl_variant_count(B.ICL_OP_CONV2D_U8)))
    assert B.icl_variant_arith(B.ICL_OP_CONV2D, len(names)) is None


def _cache_with(tmp_path, key_tail, variant):
    p = tmp_path / "cache.json"
    p.write_text('{"version": 1, "entries": [\n  {"key": "unknown|0|%s", "variant": "%s", "us": 1.0}\n]}\n'
                 % (key_tail, variant))
    return str(p)


def test_split_arithmetic_is_selected_only_after_opting_in(no_gpu, tmp_path):
    """A tuned entry that names the float16-split variant is never selected in the float32 mode:
    cache keys carry the arithmetic mode, and a selection re-checks the variant's arithmetic."""
    idx = B.variant_names(B.ICL_OP_CONV2D).index("mfma_f16x3")
    side = 4096
    sc = (side * side).bit_length() - 1
    try:
        for mode in (0, 1):   # an entry under each mode's key, both naming the split variant
            assert B.icl_tune_load(_cache_with(tmp_path, f"conv2d|0|7|{sc}|f1|m{mode}", "mfma_f16x3")) == B.ICL_OK
        st, got = B.icl_selected_variant(B.ICL_OP_CONV2D, B.ICL_F32, 7, side, side)
        assert st == B.ICL_OK and got == 1          # float32 mode: the default FMA tile
        assert B.icl_set_math(B.ICL_MATH_F16_SPLIT) == B.ICL_OK
        st, got = B.icl_selected_variant(B.ICL_OP_CONV2D, B.ICL_F32, 7, side, side)
        assert st == B.ICL_OK and got == idx        # opted in: the tuned split variant
        B.icl_tune_clear()
        assert B.icl_tune_load(_cache_with(tmp_path, f"conv2d|0|7|{sc}|f1|m0", "lds_p4x8_o0")) == B.ICL_OK
        st, got = B.icl_selected_variant(B.ICL_OP_CONV2D, B.ICL_F32, 7, side, side)
        assert got == 1                             # an entry of the other mode does not apply
    finally:
        B.icl_set_math(B.ICL_MATH_F32)
        B.icl_tune_clear()


def test_problem_tuning_validation(no_gpu):
    P = B.icl_tune_problem
    assert B.lib().icl_tune_problem(None, None) == B.ICL_ERR_INVALID_VALUE
    assert P(B.ICL_OP_CONV_SEP_BATCHED, B.ICL_F16, 2, 64, 64) == B.ICL_ERR_INVALID_VALUE   # tuned per plan
    assert P(B.ICL_OP_BANK_FWD, B.ICL_F32, 5, 64, 64, n=2, f=4) == B.ICL_ERR_RADIUS
    assert P(B.ICL_OP_BANK_FWD, B.ICL_F32, 4, 64, 64, n=2, f=65) == B.ICL_ERR_UNSUPPORTED
    assert P(B.ICL_OP_BANK_BWD_FILTER, B.ICL_F16, 4, 64, 64, n=2, f=4) == B.ICL_ERR_DTYPE
    assert P(B.ICL_OP_CONV3D_SEP, B.ICL_F32, 8, 64, 64, depth=8) == B.ICL_ERR_RADIUS
    assert P(B.ICL_OP_CONV2D, B.ICL_F32, 2, 0, 64) == B.ICL_ERR_INVALID_VALUE
    assert P(B.ICL_OP_BANK_FWD_SSE, B.ICL_F32, 4, 64, 64, n=2, f=16) == B.ICL_ERR_NO_DEVICE
    assert P(B.ICL_OP_CONV3D_SEP, B.ICL_F32, 1, 64, 64, depth=64) == B.ICL_ERR_NO_DEVICE
    # defaults of the problem form: the matrix-core forward and filter adjoint up to 16 filters
    st, v = B.icl_selected_variant_problem(B.ICL_OP_BANK_FWD, B.ICL_F32, 4, 1024, 1024, n=32, f=16)
    assert st == B.ICL_OK and B.icl_variant_name(B.ICL_OP_BANK_FWD, v) == "mfma_px_t64"
    st, v = B.icl_selected_variant_problem(B.ICL_OP_BANK_BWD_FILTER, B.ICL_F32, 4, 1024, 1024, n=32, f=32)
    assert st == B.ICL_OK and B.icl_variant_name(B.ICL_OP_BANK_BWD_FILTER, v) == "block4_t64x256"
    assert B.icl_batch_plan_tune(0) == B.ICL_ERR_INVALID_VALUE
    assert B.icl_batch_plan_variant(0)[0] == B.ICL_ERR_INVALID_VALUE


def test_tune_environment_modes(tmp_path):
    """ICL_TUNE_CACHE is loaded at the first selection; ICL_TUNE=off ignores it (fresh processes,
    since the environment is read once)."""
    import subprocess
    import sys
    side = 1024
    sc = (side * side).bit_length() - 1
    path = _cache_with(tmp_path, f"conv2d|0|3|{sc}|f1|m0", "pers_p8x2")
    code = ("import sys; sys.path.insert(0, %r); from paper_1605_06399_amd import binding as B; "
            "print(B.icl_variant_name(B.ICL_OP_CONV2D, B.icl_selected_variant(B.ICL_OP_CONV2D, B.ICL_F32, 3, %d, %d)[1]))"
            % (ROOT, side, side))
    env = dict(os.environ, ICL_TUNE_CACHE=path, HIP_VISIBLE_DEVICES="")
    for mode, want in (("cache", "pers_p8x2"), ("off", "lds_p4x4_o0")):
        out = subprocess.run([sys.executable, "-c", code], env=dict(env, ICL_TUNE=mode), capture_output=True,
                             text=True, timeout=120)
        assert out.returncode == 0, out.stderr
        assert out.stdout.strip() == want, (mode, out.stdout, out.stderr)


def test_adjoint_scale_validation(no_gpu):
    # a factor that overlaps the output is an alias; a separate one reaches the device check
    assert B.icl_bank_bwd_input(SRC, TAPS, DST, 2, 4, 8, 8, 4, scale=DST + 8) == B.ICL_ERR_ALIAS
    assert B.icl_bank_bwd_input(SRC, TAPS, DST, 2, 4, 8, 8, 4, scale=WS) == B.ICL_ERR_NO_DEVICE
    _, nb = B.icl_workspace_size(B.ICL_OP_BANK_BWD_FILTER, 8, 8, 2, 4, 4)
    assert B.icl_bank_bwd_filter(SRC, DST, 0x70000000, 2, 4, 8, 8, 4, WS, nb, scale=0x70000000 + 4) == B.ICL_ERR_ALIAS
    assert B.icl_bank_bwd_filter(SRC, DST, 0x70000000, 2, 4, 8, 8, 4, WS, nb, scale=WS + 4) == B.ICL_ERR_ALIAS
