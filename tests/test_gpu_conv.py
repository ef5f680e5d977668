"""GPU parity: separable and 2-D correlation, every variant, against the FP64 oracle.

Shapes span several tiles with ragged tails, plus degenerate images (1x1, one
row, one column, smaller than the stencil), padded pitches and misaligned
starts (which switch off the vector paths).
"""
import numpy as np
import pytest

from conftest import gpu_available
from helpers import assert_close, empty_padded, padded_view, storage, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

from oracle import oracle  # noqa: E402
from paper_1605_06399_amd import binding as B, synth  # noqa: E402

if gpu_available():
    import torch
    from paper_1605_06399_amd import torch_api as T


def _nvariants(op, default):
    try:
        return B.icl_variant_count(op)
    except Exception:
        return default


N_SEP = _nvariants(B.ICL_OP_CONV_SEP, 9)
N_2D = _nvariants(B.ICL_OP_CONV2D, 10)


@pytest.fixture
def force():
    ops = []

    def _force(op, idx):
        ops.append(op)
        B.check(B.icl_force_variant(op, idx))

    yield _force
    for op in ops:
        B.icl_force_variant(op, -1)


def taps_sep(r, cfg=40):
    h = synth.normal_taps_normalised(cfg, 2 * r + 1, stream=2 * r)
    v = synth.normal_taps_normalised(cfg, 2 * r + 1, stream=2 * r + 1)
    return h, v


def taps_2d(r, cfg=41):
    n = 2 * r + 1
    return synth.normal_taps_normalised(cfg, n * n, stream=r).reshape(n, n)


def dev_taps(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).ravel()).cuda()


SHAPES = [(389, 517), (1, 1), (1, 70), (70, 1), (3, 5), (64, 64), (33, 200)]


def sep_ws(H, W):
    _, nb = B.icl_workspace_size(B.ICL_OP_CONV_SEP, W, H)
    return torch.empty(nb // 4 + 1, dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("variant", range(N_SEP))
@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("r", [0, 1, 2, 3, 5, 7])
def test_conv_sep_variants(force, variant, dt, r):
    if variant >= B.icl_variant_count(B.ICL_OP_CONV_SEP):
        pytest.skip("no such variant")
    force(B.ICL_OP_CONV_SEP, variant)
    h, v = taps_sep(r)
    for (H, W) in SHAPES:
        img = synth.image_uniform(42, H, W)
        xd, x64 = storage(img, dt)
        out = T.conv_sep(xd, dev_taps(h), dev_taps(v), workspace=sep_ws(H, W))
        torch.cuda.synchronize()
        ref = oracle.conv_sep(x64, h, v)
        assert_close(out, ref, oracle.normwise_scale_sep(x64, h, v), dt, f"sep v{variant} {dt} r{r} {H}x{W}")


@pytest.mark.parametrize("variant", range(N_2D))
@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("r", [0, 1, 2, 3, 5, 7])
def test_conv2d_variants(force, variant, dt, r):
    if variant >= B.icl_variant_count(B.ICL_OP_CONV2D):
        pytest.skip("no such variant")
    force(B.ICL_OP_CONV2D, variant)
    w = taps_2d(r)
    for (H, W) in SHAPES:
        img = synth.image_uniform(43, H, W)
        xd, x64 = storage(img, dt)
        out = T.conv2d(xd, dev_taps(w).view(w.shape))
        torch.cuda.synchronize()
        ref = oracle.conv2d(x64, w)
        assert_close(out, ref, oracle.normwise_scale_conv2d(x64, w), dt, f"2d v{variant} {dt} r{r} {H}x{W}")


@pytest.mark.parametrize("r", [9, 16])
def test_large_radius_plain_paths(r):
    """Radii above the templated range run the runtime-radius plain kernels (sep needs its workspace)."""
    H, W = 45, 77
    img = synth.image_uniform(44, H, W)
    h, v = taps_sep(r)
    w = taps_2d(r)
    xd, x64 = storage(img, "f32")
    out = T.conv_sep(xd, dev_taps(h), dev_taps(v))
    out2 = T.conv2d(xd, dev_taps(w).view(w.shape))
    torch.cuda.synchronize()
    assert_close(out, oracle.conv_sep(x64, h, v), oracle.normwise_scale_sep(x64, h, v), "f32", "sep r>7")
    assert_close(out2, oracle.conv2d(x64, w), oracle.normwise_scale_conv2d(x64, w), "f32", "2d r>7")
    # without a workspace the separable call must refuse, not fall back silently
    sp = xd.data_ptr()
    st = B.icl_conv_sep(sp, W * 4, out.data_ptr(), W * 4, W, H, B.ICL_F32, dev_taps(h).data_ptr(),
                        dev_taps(v).data_ptr(), r, 0, 0, 0)
    assert st == B.ICL_ERR_WORKSPACE


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("pad,off", [(3, 1), (37, 0), (64, 2)])
def test_padded_pitch_and_misaligned(dt, pad, off):
    H, W, r = 70, 131, 3
    img = synth.image_uniform(45, H, W)
    xd, x64 = storage(img, dt)
    xv = padded_view(xd, pad, off)
    h, v = taps_sep(r)
    w = taps_2d(r)
    for variant_op, fn in ((B.ICL_OP_CONV_SEP, "sep"), (B.ICL_OP_CONV2D, "2d")):
        for variant in range(B.icl_variant_count(variant_op)):
            B.check(B.icl_force_variant(variant_op, variant))
            try:
                out = empty_padded(H, W, xd.dtype, pad + 5, off + 1)
                if fn == "sep":
                    T.conv_sep(xv, dev_taps(h), dev_taps(v), out=out, workspace=sep_ws(H, W))
                    ref, sc = oracle.conv_sep(x64, h, v), oracle.normwise_scale_sep(x64, h, v)
                else:
                    T.conv2d(xv, dev_taps(w).view(w.shape), out=out)
                    ref, sc = oracle.conv2d(x64, w), oracle.normwise_scale_conv2d(x64, w)
                torch.cuda.synchronize()
                assert_close(out, ref, sc, dt, f"{fn} v{variant} pad{pad} off{off}")
            finally:
                B.icl_force_variant(variant_op, -1)


def test_delta_and_integer_masks_bit_exact():
    """Delta filters reproduce the input, and small integer masks on integer images are exact in
    float32 whatever the summation order, so every variant must match the oracle bit for bit."""
    H, W = 133, 257
    img = synth.integer_image(46, H, W)
    xd, x64 = storage(img, "f32")
    b = np.array([1, 4, 6, 4, 1], np.float32)
    box = np.ones((3, 3), np.float32)
    for r in (1, 2, 3):
        d = np.zeros(2 * r + 1, np.float32)
        d[r] = 1
        for variant in range(B.icl_variant_count(B.ICL_OP_CONV_SEP)):
            B.check(B.icl_force_variant(B.ICL_OP_CONV_SEP, variant))
            out = T.conv_sep(xd, dev_taps(d), dev_taps(d), workspace=sep_ws(H, W))
            assert np.array_equal(to_host(out), x64)
        B.icl_force_variant(B.ICL_OP_CONV_SEP, -1)
    for variant in range(B.icl_variant_count(B.ICL_OP_CONV_SEP)):
        B.check(B.icl_force_variant(B.ICL_OP_CONV_SEP, variant))
        out = T.conv_sep(xd, dev_taps(b), dev_taps(b), workspace=sep_ws(H, W))
        assert np.array_equal(to_host(out), oracle.conv_sep(x64, b, b))
        bn = b / 16
        out = T.conv_sep(xd, dev_taps(bn), dev_taps(bn), workspace=sep_ws(H, W))
        assert np.array_equal(to_host(out), oracle.conv_sep(x64, bn, bn))
    B.icl_force_variant(B.ICL_OP_CONV_SEP, -1)
    for variant in range(B.icl_variant_count(B.ICL_OP_CONV2D)):
        B.check(B.icl_force_variant(B.ICL_OP_CONV2D, variant))
        for w in (np.outer(b, b), box):
            out = T.conv2d(xd, dev_taps(w).view(w.shape))
            assert np.array_equal(to_host(out), oracle.conv2d(x64, w))
        d = np.zeros((5, 5), np.float32)
        d[2, 2] = 1
        assert np.array_equal(to_host(T.conv2d(xd, dev_taps(d).view(5, 5))), x64)
    B.icl_force_variant(B.ICL_OP_CONV2D, -1)


def test_taps_updated_in_place_are_seen():
    H, W, r = 50, 70, 2
    img = synth.image_uniform(47, H, W)
    xd, x64 = storage(img, "f32")
    g = synth.gaussian_taps(r, 1.0)
    t = dev_taps(g)
    out1 = to_host(T.conv_sep(xd, t, t))
    t.copy_(dev_taps(g[::-1] * 2))
    out2 = to_host(T.conv_sep(xd, t, t))
    assert np.allclose(out2, 4 * out1, rtol=1e-6)


def test_tuner_selects_a_valid_variant(tmp_path):
    H, W = 512, 512
    for op, r in ((B.ICL_OP_CONV_SEP, 2), (B.ICL_OP_CONV2D, 3)):
        B.check(B.icl_tune(op, B.ICL_F32, r, W, H), "tune")
        st, idx = B.icl_selected_variant(op, B.ICL_F32, r, W, H)
        assert st == B.ICL_OK and idx >= 1
        img = synth.image_uniform(48, H, W)
        xd, x64 = storage(img, "f32")
        if op == B.ICL_OP_CONV_SEP:
            h, v = taps_sep(r)
            out = T.conv_sep(xd, dev_taps(h), dev_taps(v))
            ref, sc = oracle.conv_sep(x64, h, v), oracle.normwise_scale_sep(x64, h, v)
        else:
            w = taps_2d(r)
            out = T.conv2d(xd, dev_taps(w).view(w.shape))
            ref, sc = oracle.conv2d(x64, w), oracle.normwise_scale_conv2d(x64, w)
        torch.cuda.synchronize()
        assert_close(out, ref, sc, "f32", f"tuned op {op}")
    p = tmp_path / "tune.json"
    assert B.icl_tune_save(str(p)) == B.ICL_OK
    B.icl_tune_clear()
    assert B.icl_tune_load(str(p)) == B.ICL_OK
    st, idx = B.icl_selected_variant(B.ICL_OP_CONV2D, B.ICL_F32, 3, W, H)
    assert idx >= 1
    B.icl_tune_clear()


def _mfma_index():
    names = B.variant_names(B.ICL_OP_CONV2D)
    return names.index("mfma_f16x3") if "mfma_f16x3" in names else None


@pytest.mark.parametrize("r", [3, 7])
@pytest.mark.parametrize("img_exp,tap_exp", [(60, 0), (-60, 0), (0, 40), (-100, -20), (90, 20)])
def test_mfma_variant_power_of_two_scaling(force, r, img_exp, tap_exp):
    """The matrix-core variant scales each tile and the taps by powers of two: inputs far from
    float16's range give the same normwise error as unit-range ones."""
    idx = _mfma_index()
    if idx is None:
        pytest.skip("no matrix-core variant")
    force(B.ICL_OP_CONV2D, idx)
    H, W = 150, 210
    img = np.ldexp(synth.image_uniform(49, H, W).astype(np.float64) - 0.5, img_exp).astype(np.float32)
    w = np.ldexp(taps_2d(r).astype(np.float64), tap_exp).astype(np.float32)
    xd, x64 = storage(img, "f32")
    out = T.conv2d(xd, dev_taps(w).view(w.shape))
    torch.cuda.synchronize()
    w64 = w.astype(np.float64)
    assert_close(out, oracle.conv2d(x64, w64), oracle.normwise_scale_conv2d(x64, w64), "f32", f"mfma 2^{img_exp} 2^{tap_exp}")


def _wide_contrast(seed, H, W):
    """U[0,1) image whose right half is scaled by 2^-30: windows there sit 2^30 below the
    brightest pixel of tiles that straddle the step."""
    img = synth.image_uniform(seed, H, W).astype(np.float64)
    img[:, W // 2:] *= 2.0 ** -30
    return img.astype(np.float32)


@pytest.mark.parametrize("r", [2, 5, 7])
def test_float32_mode_variants_meet_1e5_at_wide_contrast(force, r):
    """In the default float32 arithmetic mode the tuner may pick every variant but the float16
    split one; each of them meets the float32 normwise tolerance 1e-5 on an image spanning 2^30
    in contrast, and the tuner's choice is one of them."""
    assert B.icl_get_math() == B.ICL_MATH_F32
    H, W = 130, 200
    img = _wide_contrast(50, H, W)
    w = taps_2d(r)
    xd, x64 = storage(img, "f32")
    w64 = w.astype(np.float64)
    ref, S = oracle.conv2d(x64, w64), oracle.normwise_scale_conv2d(x64, w64)
    for i in range(B.icl_variant_count(B.ICL_OP_CONV2D)):
        if B.icl_variant_arith(B.ICL_OP_CONV2D, i) == "fp16x3_mfma":
            continue
        force(B.ICL_OP_CONV2D, i)
        out = T.conv2d(xd, dev_taps(w).view(w.shape))
        torch.cuda.synchronize()
        assert_close(out, ref, S, "f32", f"variant {i} r{r} at 2^-30 contrast")
    B.icl_force_variant(B.ICL_OP_CONV2D, -1)
    try:
        B.check(B.icl_tune(B.ICL_OP_CONV2D, B.ICL_F32, r, 1024, 1024), "tune")
        st, idx = B.icl_selected_variant(B.ICL_OP_CONV2D, B.ICL_F32, r, 1024, 1024)
        assert st == B.ICL_OK and B.icl_variant_arith(B.ICL_OP_CONV2D, idx) == "fp32_valu"
    finally:
        B.icl_tune_clear()


@pytest.mark.parametrize("r", [2, 7])
def test_mfma_variant_wide_range_bound(force, r):
    """The float16-split variant runs only when forced or after opting into ICL_MATH_F16_SPLIT,
    whose stated accuracy it is tested against here: dark regions 2^-30 below a bright one in
    the same tile stay within the operand bound 2^-20 S + 2^-37 (2r+1)^2 M max|w| (plus the
    float32 accumulation allowance 1e-5 S of every variant)."""
    idx = _mfma_index()
    if idx is None:
        pytest.skip("no matrix-core variant")
    force(B.ICL_OP_CONV2D, idx)
    H, W = 130, 200
    img = _wide_contrast(50, H, W)
    w = taps_2d(r)
    xd, x64 = storage(img, "f32")
    out = to_host(T.conv2d(xd, dev_taps(w).view(w.shape)))
    w64 = w.astype(np.float64)
    ref = oracle.conv2d(x64, w64)
    S = oracle.normwise_scale_conv2d(x64, w64)
    M = float(np.abs(x64).max())
    bound = 1e-5 * S + 2.0 ** -20 * S + 2.0 ** -37 * (2 * r + 1) ** 2 * M * float(np.abs(w64).max())
    assert np.all(np.abs(out - ref) <= bound)


def test_split_mode_opt_in_tunes_every_candidate():
    """After opting into ICL_MATH_F16_SPLIT the tuner's candidates include the split variant; the
    choice is cached under that mode only, and going back to float32 never selects it."""
    W = H = 1024
    try:
        B.check(B.icl_set_math(B.ICL_MATH_F16_SPLIT))
        B.check(B.icl_tune(B.ICL_OP_CONV2D, B.ICL_F32, 7, W, H), "tune split mode")
        st, idx_split = B.icl_selected_variant(B.ICL_OP_CONV2D, B.ICL_F32, 7, W, H)
        assert st == B.ICL_OK and idx_split >= 1
        B.check(B.icl_set_math(B.ICL_MATH_F32))
        st, idx = B.icl_selected_variant(B.ICL_OP_CONV2D, B.ICL_F32, 7, W, H)
        assert B.icl_variant_arith(B.ICL_OP_CONV2D, idx) == "fp32_valu"
    finally:
        B.icl_set_math(B.ICL_MATH_F32)
        B.icl_tune_clear()


def test_single_image_512_gaussian_whole_image(force):
    """The single-image workload: 512^2 float32 U[0,1) (seed config 1), the 5-tap Gaussian sigma = 1
    in both passes, clamped; the plain two-pass kernel, every fused variant and the tuned choice
    against the oracle over the whole image."""
    H = W = 512
    img = synth.image_uniform(1, H, W)
    g = synth.gaussian_taps(2, 1.0)
    xd, x64 = storage(img, "f32")
    ref, sc = oracle.conv_sep(x64, g, g), oracle.normwise_scale_sep(x64, g, g)
    _, nb = B.icl_workspace_size(B.ICL_OP_CONV_SEP, W, H)
    ws = torch.empty(nb // 4 + 1, dtype=torch.float32, device="cuda")
    tg = dev_taps(g)
    for i in range(B.icl_variant_count(B.ICL_OP_CONV_SEP)):
        force(B.ICL_OP_CONV_SEP, i)
        out = T.conv_sep(xd, tg, tg, workspace=ws)
        torch.cuda.synchronize()
        assert_close(out, ref, sc, "f32", f"512^2 gaussian, variant {i}")
    B.icl_force_variant(B.ICL_OP_CONV_SEP, -1)
    try:
        B.check(B.icl_tune(B.ICL_OP_CONV_SEP, B.ICL_F32, 2, W, H), "tune")
        out = T.conv_sep(xd, tg, tg, workspace=ws)
        torch.cuda.synchronize()
        assert_close(out, ref, sc, "f32", "512^2 gaussian, tuned")
    finally:
        B.icl_tune_clear()
