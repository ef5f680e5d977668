"""GPU parity: fused corner detection (Harris response + 3x3 NMS in one pass).

Every variant runs with the response written too, so that two exact checks apply:
  * the mask is the oracle's NMS of the kernel's own response, bit for bit (the NMS
    decision takes float32 values, which double holds exactly);
  * the response matches the oracle's Harris response within the oracle's bound on the
    rounding error of a float32 evaluation of the chain.
The single-pass variants must also agree with each other byte for byte (mask) and bit for
bit (response), with and without the response output, and on padded or misaligned images.
"""
import numpy as np
import pytest

from conftest import gpu_available
from helpers import normwise, padded_view, storage, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

from oracle import oracle  # noqa: E402
from paper_1605_06399_amd import binding as B, synth  # noqa: E402

if gpu_available():
    import torch
    from paper_1605_06399_amd import torch_api as T

K = np.float32(0.04)
TAU = np.float32(1e-3)
# degenerate images, narrower than a strip, one and two strips with ragged ends, ragged row
# blocks, aligned widths that reach the interior strips
SHAPES = [(1, 1), (2, 3), (5, 4), (1, 90), (90, 1), (64, 64), (17, 130), (389, 517), (133, 1100),
          (5, 700), (70, 256), (37, 752), (100, 1024), (41, 483), (300, 1024)]


def g_taps(rg):
    return synth.gaussian_taps(rg, max(rg, 1) / 2.0 if rg != 2 else 1.0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def corner_image(seed, H, W):
    return synth.image_with_rectangles(seed, H, W, count=6) if H > 16 and W > 16 else synth.image_uniform(seed, H, W)


def check_against_oracle(img64, g, R, M, what):
    Rr = oracle.harris(img64, g, float(K))
    err = normwise(to_host(R), Rr, oracle.harris_f32_bound(img64, g, float(K)))
    assert err <= 1.0, f"{what}: response error {err:.3f} x the float32 bound"
    own = oracle.nms(to_host(R), float(TAU))
    got = M.cpu().numpy()
    assert np.array_equal(got, own), f"{what}: mask differs from NMS of its own response at {np.argwhere(got != own)[:5]}"


@pytest.mark.parametrize("variant", range(6))
@pytest.mark.parametrize("rg", [0, 1, 2, 3])
def test_corners_variants(variant, rg):
    if variant >= B.icl_variant_count(B.ICL_OP_CORNERS):
        pytest.skip("no such variant")
    B.check(B.icl_force_variant(B.ICL_OP_CORNERS, variant))
    try:
        g = g_taps(rg)
        for (H, W) in SHAPES:
            xd, x64 = storage(corner_image(50 + rg, H, W), "f32")
            R = torch.full((H, W), float("nan"), dtype=torch.float32, device="cuda")
            M = T.corners(xd, dev(g), float(K), float(TAU), resp=R)
            torch.cuda.synchronize()
            check_against_oracle(x64, g, R, M, f"v{variant} rg{rg} {H}x{W}")
            if variant > 0:   # the mask alone: the same pass without the response store
                M2 = T.corners(xd, dev(g), float(K), float(TAU))
                assert torch.equal(M, M2), f"v{variant} rg{rg} {H}x{W}: mask changes without the response output"
    finally:
        B.icl_force_variant(B.ICL_OP_CORNERS, -1)


@pytest.mark.parametrize("rg", [1, 2, 3])
def test_single_pass_variants_agree_bitwise(rg):
    H, W = 301, 1000
    g = g_taps(rg)
    xd, _ = storage(corner_image(55, H, W), "f32")
    outs = []
    for variant in range(1, B.icl_variant_count(B.ICL_OP_CORNERS)):
        B.check(B.icl_force_variant(B.ICL_OP_CORNERS, variant))
        try:
            R = torch.empty((H, W), dtype=torch.float32, device="cuda")
            M = T.corners(xd, dev(g), float(K), float(TAU), resp=R)
            outs.append((variant, M, R))
        finally:
            B.icl_force_variant(B.ICL_OP_CORNERS, -1)
    for v, M, R in outs[1:]:
        assert torch.equal(M, outs[0][1]), f"mask of variant {v}"
        assert torch.equal(R.view(torch.int32), outs[0][2].view(torch.int32)), f"response of variant {v}"


@pytest.mark.parametrize("pad,off,moff", [(3, 1, 1), (37, 0, 3), (64, 2, 0)])
def test_corners_padded_and_misaligned(pad, off, moff):
    """Misaligned image rows switch off the vector loads; odd mask pitches the word stores."""
    H, W, rg = 77, 611, 2
    g = g_taps(rg)
    xd, x64 = storage(corner_image(56, H, W), "f32")
    xv = padded_view(xd, pad, off)
    for variant in range(B.icl_variant_count(B.ICL_OP_CORNERS)):
        B.check(B.icl_force_variant(B.ICL_OP_CORNERS, variant))
        try:
            mbuf = torch.full(((H + 1) * (W + pad + 3) + moff + 16,), 0xA5, dtype=torch.uint8, device="cuda")
            M = mbuf[moff:moff + H * (W + pad + 3)].view(H, W + pad + 3)[:, :W]
            R = torch.empty((H, W + 5), dtype=torch.float32, device="cuda")[:, :W]
            T.corners(xv, dev(g), float(K), float(TAU), out=M, resp=R)
            torch.cuda.synchronize()
            check_against_oracle(x64, g, R, M, f"v{variant} pad{pad} off{off} moff{moff}")
            full = mbuf.cpu().numpy()
            keep = np.ones(full.shape, bool)
            for y in range(H):
                s0 = moff + y * (W + pad + 3)
                keep[s0:s0 + W] = False
            assert np.all(full[keep] == 0xA5), f"v{variant} wrote outside the mask image"
        finally:
            B.icl_force_variant(B.ICL_OP_CORNERS, -1)


def test_corners_other_radii_and_workspace():
    """NMS radius 2 and window radius 5 run the two kernels: through the caller's response
    image, through the workspace, and not at all without either."""
    H, W = 90, 333
    xd, x64 = storage(corner_image(57, H, W), "f32")
    for rg, nr in ((2, 2), (5, 1)):
        g = g_taps(rg)
        R = torch.empty((H, W), dtype=torch.float32, device="cuda")
        _, nbs = B.icl_workspace_size(B.ICL_OP_CORNERS, W, H, radius=rg)
        wsr = torch.empty(nbs // 4 + 1, dtype=torch.float32, device="cuda")
        M = T.corners(xd, dev(g), float(K), float(TAU), nms_radius=nr, resp=R, workspace=wsr)
        torch.cuda.synchronize()
        assert np.array_equal(M.cpu().numpy(), oracle.nms(to_host(R), float(TAU), radius=nr))
        _, nb = B.icl_workspace_size(B.ICL_OP_CORNERS, W, H, radius=rg)
        assert nb >= W * H * 4 + (2 * W * H * 4 if rg > 3 else 0)
        ws = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
        M2 = T.corners(xd, dev(g), float(K), float(TAU), nms_radius=nr, workspace=ws)
        assert torch.equal(M, M2)
        if rg > 3:   # the response given, the gradient images still from the workspace
            _, nb3 = B.icl_workspace_size(B.ICL_OP_CORNERS, W, H, radius=rg)
            M3 = T.corners(xd, dev(g), float(K), float(TAU), nms_radius=nr, resp=torch.empty_like(R),
                           workspace=ws)
            assert torch.equal(M, M3)
        out = torch.empty_like(M)
        st = B.icl_corners(xd.data_ptr(), W * 4, out.data_ptr(), W, W, H, dev(g).data_ptr(), rg, float(K), nr,
                           float(TAU), 0, 0, 0, 0, torch.cuda.current_stream().cuda_stream)
        assert st == B.ICL_ERR_WORKSPACE


def test_fused_matches_two_calls_inside_the_strips():
    """Inside the strip regions both paths evaluate the same float32 expression for R, so the
    fused mask equals icl_harris followed by icl_nms there, byte for byte."""
    H, W, rg = 512, 2048, 2
    g = g_taps(rg)
    xd, _ = storage(corner_image(58, H, W), "f32")
    M = T.corners(xd, dev(g), float(K), float(TAU))
    R2 = T.harris(xd, dev(g), float(K))
    M2 = T.nms(R2, float(TAU))
    xr = 4 + ((W - 8) // 248) * 248        # the separate Harris strips cover columns [4, xr)
    a, b = M[:, 8:xr - 8], M2[:, 8:xr - 8]
    assert torch.equal(a, b), f"{int((a != b).sum())} mask bytes differ"


def test_tuner_corners():
    H, W = 256, 1024
    try:
        B.check(B.icl_tune(B.ICL_OP_CORNERS, B.ICL_F32, 2, W, H), "tune corners")
        st, idx = B.icl_selected_variant(B.ICL_OP_CORNERS, B.ICL_F32, 2, W, H)
        assert st == B.ICL_OK and idx >= 1
        g = g_taps(2)
        xd, x64 = storage(corner_image(59, H, W), "f32")
        R = torch.empty((H, W), dtype=torch.float32, device="cuda")
        M = T.corners(xd, dev(g), float(K), float(TAU), resp=R)
        check_against_oracle(x64, g, R, M, "tuned")
    finally:
        B.icl_tune_clear()
