"""GPU parity: Harris response and non-maximum suppression against the FP64 oracle."""
import numpy as np
import pytest

from conftest import gpu_available
from helpers import empty_padded, nms_ambiguous, normwise, padded_view, storage, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

from oracle import oracle  # noqa: E402
from paper_1605_06399_amd import binding as B, synth  # noqa: E402

if gpu_available():
    import torch
    from paper_1605_06399_amd import torch_api as T

K = np.float32(0.04)
TAU = np.float32(1e-3)


def g_taps(rg):
    return synth.gaussian_taps(rg, max(rg, 1) / 2.0 if rg != 2 else 1.0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def harris_ws(H, W):
    _, nb = B.icl_workspace_size(B.ICL_OP_HARRIS, W, H)
    return torch.empty(nb // 4 + 1, dtype=torch.float32, device="cuda")


def _nvariants(op, default):
    try:
        return B.icl_variant_count(op)
    except Exception:
        return default


N_HARRIS = _nvariants(B.ICL_OP_HARRIS, 7)
STREAM_MIN_W = 4 + 248 + 4     # the strip variants need one strip between the two border bands


def runs(variant, W):
    """Whether a forced variant accepts a dense W-wide image: the strip variants need
    W >= STREAM_MIN_W and 16-byte aligned rows (W a multiple of 4 here)."""
    return not B.icl_variant_name(B.ICL_OP_HARRIS, variant).startswith("stream") or (
        W >= STREAM_MIN_W and W % 4 == 0)


# small and degenerate images, several strips with a ragged right band and ragged row
# blocks, fewer rows than a row block, one row, and the narrowest width the strips take
HARRIS_SHAPES = [(389, 517), (1, 1), (2, 3), (5, 4), (1, 90), (90, 1), (64, 64), (17, 130),
                 (133, 1100), (5, 700), (1, 640), (300, STREAM_MIN_W), (70, STREAM_MIN_W + 4), (37, 752)]


@pytest.mark.parametrize("variant", range(N_HARRIS))
@pytest.mark.parametrize("rg", [0, 1, 2, 3])
def test_harris_variants(variant, rg):
    if variant >= B.icl_variant_count(B.ICL_OP_HARRIS):
        pytest.skip("no such variant")
    B.check(B.icl_force_variant(B.ICL_OP_HARRIS, variant))
    try:
        g = g_taps(rg)
        for (H, W) in HARRIS_SHAPES:
            if not runs(variant, W):
                continue
            img = synth.image_with_rectangles(49, H, W, count=6) if H > 16 else synth.image_uniform(49, H, W)
            xd, x64 = storage(img, "f32")
            R = T.harris(xd, dev(g), float(K), workspace=harris_ws(H, W))
            torch.cuda.synchronize()
            Rr = oracle.harris(x64, g, float(K))
            err = normwise(to_host(R), Rr, oracle.harris_f32_bound(x64, g, float(K)))
            assert err <= 1.0, f"harris v{variant} rg{rg} {H}x{W}: error {err:.3f} x the float32 bound"
    finally:
        B.icl_force_variant(B.ICL_OP_HARRIS, -1)


def test_harris_large_window_uses_split_path():
    H, W, rg = 60, 75, 5
    g = synth.gaussian_taps(rg, 2.5)
    img = synth.image_uniform(50, H, W)
    xd, x64 = storage(img, "f32")
    R = T.harris(xd, dev(g), float(K))
    torch.cuda.synchronize()
    Rr = oracle.harris(x64, g, float(K))
    assert normwise(to_host(R), Rr, oracle.harris_f32_bound(x64, g, float(K))) <= 1.0


@pytest.mark.parametrize("variant", range(N_HARRIS))
def test_harris_closed_forms_on_gpu(variant):
    if variant >= B.icl_variant_count(B.ICL_OP_HARRIS):
        pytest.skip("no such variant")
    B.check(B.icl_force_variant(B.ICL_OP_HARRIS, variant))
    try:
        g = synth.gaussian_taps(2, 1.0)
        H, W = 70, 90 if runs(variant, 90) else STREAM_MIN_W + 12
        # constant image: every gradient is exactly zero, so R is exactly zero
        R = T.harris(torch.full((H, W), 0.3, device="cuda"), dev(g), float(K), workspace=harris_ws(H, W))
        assert torch.count_nonzero(R).item() == 0
        # linear ramp I = x + 2y (exact in float32): R = -k (64 * 5)^2 * (sum g)^4 away from the edges
        y, x = np.meshgrid(np.arange(H, dtype=np.float32), np.arange(W, dtype=np.float32), indexing="ij")
        R = to_host(T.harris(dev(x + 2 * y), dev(g), float(K), workspace=harris_ws(H, W)))
        s = float(np.sum(g.astype(np.float64)))
        expect = -float(K) * (64.0 * 5.0 * s * s) ** 2
        assert np.allclose(R[3:-3, 3:-3], expect, rtol=2e-6)
    finally:
        B.icl_force_variant(B.ICL_OP_HARRIS, -1)


def test_harris_strip_variants_refuse_unaligned_rows():
    """A forced strip variant needs 16-byte aligned rows; automatic selection falls back."""
    H, W = 40, 600
    img = synth.image_uniform(53, H, W)
    xd, x64 = storage(img, "f32")
    xv = padded_view(xd, 3, 1)
    g = synth.gaussian_taps(2, 1.0)
    ref = oracle.harris(x64, g, float(K))
    for v in range(B.icl_variant_count(B.ICL_OP_HARRIS)):
        if not B.icl_variant_name(B.ICL_OP_HARRIS, v).startswith("stream"):
            continue
        B.check(B.icl_force_variant(B.ICL_OP_HARRIS, v))
        try:
            with pytest.raises(B.IclError):
                T.harris(xv, dev(g), float(K))
        finally:
            B.icl_force_variant(B.ICL_OP_HARRIS, -1)
    R = T.harris(xv, dev(g), float(K))
    torch.cuda.synchronize()
    assert normwise(to_host(R), ref, oracle.harris_f32_bound(x64, g, float(K))) <= 1.0
    # an odd width in rows padded to a 16-byte pitch: the strips take it
    H, W = 45, 517
    img = synth.image_with_rectangles(54, H, W, count=5)
    xd, x64 = storage(img, "f32")
    xv = padded_view(xd, 3, 0)
    out = empty_padded(H, W, torch.float32, 7, 0)
    ref, sc = oracle.harris(x64, g, float(K)), oracle.harris_f32_bound(x64, g, float(K))
    for v in range(B.icl_variant_count(B.ICL_OP_HARRIS)):
        if not B.icl_variant_name(B.ICL_OP_HARRIS, v).startswith("stream"):
            continue
        B.check(B.icl_force_variant(B.ICL_OP_HARRIS, v))
        try:
            R = T.harris(xv, dev(g), float(K), out=out)
            torch.cuda.synchronize()
            assert normwise(to_host(R), ref, sc) <= 1.0, f"variant {v} padded pitch"
        finally:
            B.icl_force_variant(B.ICL_OP_HARRIS, -1)


def quantised_response(H, W, seed):
    """Synthetic responses with many exact ties, plateaus and values at the threshold."""
    u = synth.uniform01(synth.seed(seed, 0), H * W).reshape(H, W)
    q = (np.floor(u * 6) - 1).astype(np.float32) * np.float32(1e-3)   # {-1e-3, 0, 1e-3, .. 4e-3}
    q[q == np.float32(1e-3)] = TAU                                   # exactly tau: never above threshold
    return q


N_NMS = _nvariants(B.ICL_OP_NMS, 4)


def nms_runs(variant, radius, W, aligned=True):
    """Whether a forced NMS variant takes the input: row4 needs r = 1; the strip variants need
    r = 1, W >= STREAM_MIN_W and 16-byte aligned response rows (dense: W a multiple of 4)."""
    name = B.icl_variant_name(B.ICL_OP_NMS, variant)
    if name == "row4":
        return radius == 1
    if name.startswith("stream"):
        return radius == 1 and W >= STREAM_MIN_W and aligned
    return True


NMS_SHAPES = [(257, 389), (1, 1), (1, 9), (9, 1), (4, 4), (63, 65),
              (133, 1100), (5, 700), (1, 640), (300, STREAM_MIN_W), (70, STREAM_MIN_W + 4), (129, 2000), (37, 752)]


@pytest.mark.parametrize("variant", range(N_NMS))
@pytest.mark.parametrize("radius", [1, 2])
def test_nms_bit_exact(variant, radius):
    if variant >= B.icl_variant_count(B.ICL_OP_NMS):
        pytest.skip("no such variant")
    B.check(B.icl_force_variant(B.ICL_OP_NMS, variant))
    try:
        for (H, W) in NMS_SHAPES:
            R = quantised_response(H, W, 51)
            Rd = dev(R)
            st = B.icl_nms(Rd.data_ptr(), W * 4, 0, 0, W, H, radius, float(TAU), 0)   # null mask is rejected
            assert st == B.ICL_ERR_INVALID_VALUE
            if not nms_runs(variant, radius, W, W % 4 == 0):
                with pytest.raises(B.IclError):      # a forced variant never falls back silently
                    T.nms(Rd, float(TAU), radius)
                continue
            M = T.nms(Rd, float(TAU), radius)
            torch.cuda.synchronize()
            ref = oracle.nms(R, float(TAU), radius)
            assert np.array_equal(M.cpu().numpy(), ref), f"nms v{variant} r{radius} {H}x{W}"
        # padded / misaligned views take the scalar edges (the strips refuse misaligned rows)
        for (H, W, pad, off, mpad, moff) in [(70, 133, 7, 1, 7, 3), (90, 517, 3, 0, 3, 0)]:
            R = quantised_response(H, W, 52)
            Rv = padded_view(dev(R), pad, off)
            buf = torch.zeros((H + 1) * (W + mpad) + moff + 8, dtype=torch.uint8, device="cuda")
            out = buf[moff:moff + H * (W + mpad)].view(H, W + mpad)[:, :W]
            aligned = (W + pad) % 4 == 0 and off % 4 == 0 and (W + mpad) % 4 == 0 and moff % 4 == 0
            if not nms_runs(variant, radius, W, aligned):
                with pytest.raises(B.IclError):
                    T.nms(Rv, float(TAU), radius, out=out)
                continue
            M = T.nms(Rv, float(TAU), radius, out=out)
            assert np.array_equal(M.cpu().numpy(), oracle.nms(R, float(TAU), radius)), f"padded {H}x{W}"
    finally:
        B.icl_force_variant(B.ICL_OP_NMS, -1)


def test_harris_nms_pipeline_masks_agree_away_from_ties():
    """Corner masks from GPU responses vs oracle responses.  Where float rounding may decide the
    mask (R within its float32 error bound of tau or of a neighbour) both answers are correct;
    everywhere else the masks must be identical.  The bound leaves under 1% of pixels open."""
    H, W = 600, 500
    img = synth.image_with_rectangles(3, H, W, count=12)
    g = synth.gaussian_taps(2, 1.0)
    xd, x64 = storage(img, "f32")
    R = T.harris(xd, dev(g), float(K))
    M = T.nms(R, float(TAU))
    torch.cuda.synchronize()
    Rr = oracle.harris(x64, g, float(K))
    D = oracle.harris_f32_bound(x64, g, float(K))
    assert normwise(to_host(R), Rr, D) <= 1.0
    ref = oracle.nms(Rr, float(TAU))
    amb = nms_ambiguous(Rr, D, float(TAU))
    got = M.cpu().numpy()
    assert ref.sum() > 20
    assert np.array_equal(got[~amb], ref[~amb]), f"{np.sum(got[~amb] != ref[~amb])} unambiguous mismatches"
    frac = float(amb.mean())
    print(f"pipeline: {ref.sum()} corners, {amb.sum()} ambiguous pixels ({100 * frac:.2f}%)")
    assert frac <= 0.01, f"{100 * frac:.2f}% of pixels ambiguous"
