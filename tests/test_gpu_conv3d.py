"""GPU parity: separable 3-D correlation of volumes, every variant, against the FP64 oracle."""
import numpy as np
import pytest

from conftest import gpu_available
from helpers import assert_close, storage

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

from oracle import oracle  # noqa: E402
from paper_1605_06399_amd import binding as B, synth  # noqa: E402

if gpu_available():
    import torch
    from paper_1605_06399_amd import torch_api as T

# (D, H, W): degenerate, thinner than a z block, ragged x/y tiles, several z blocks
VOLUMES = [(1, 1, 1), (1, 5, 7), (3, 1, 70), (7, 19, 33), (20, 17, 130), (40, 33, 65), (70, 20, 64)]


def _nvariants(op, default):
    try:
        return B.icl_variant_count(op)
    except Exception:
        return default


N_3D = _nvariants(B.ICL_OP_CONV3D_SEP, 8)


def volume(seed, D, H, W):
    return synth.uniform01(synth.seed(seed, 0), D * H * W).reshape(D, H, W).astype(np.float32)


def taps(seed, r):
    return [synth.normal_taps_normalised(seed, 2 * r + 1, stream=q) for q in range(3)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def ws3(D, H, W):
    _, nb = B.icl_workspace_size(B.ICL_OP_CONV3D_SEP, W, H, n=D)
    return torch.empty(nb // 4 + 1, dtype=torch.float32, device="cuda")


def storage3(vol, dt):
    D, H, W = vol.shape
    xd, x64 = storage(vol.reshape(D * H, W), dt)
    return xd.view(D, H, W), x64.reshape(D, H, W)


@pytest.mark.parametrize("variant", range(N_3D))
@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_conv3d_variants(variant, dt, r):
    if variant >= B.icl_variant_count(B.ICL_OP_CONV3D_SEP):
        pytest.skip("no such variant")
    B.check(B.icl_force_variant(B.ICL_OP_CONV3D_SEP, variant))
    try:
        hx, hy, hz = taps(70 + r, r)
        for (D, H, W) in VOLUMES:
            xd, x64 = storage3(volume(71, D, H, W), dt)
            for border, c in (("clamp", 0.0), ("constant", 0.0), ("constant", 0.6)):
                out = T.conv3d_sep(xd, dev(hx), dev(hy), dev(hz), workspace=ws3(D, H, W), border=border, constant=c)
                torch.cuda.synchronize()
                ref = oracle.conv3d_sep(x64, hx, hy, hz, border=border, constant=c)
                sc = oracle.normwise_scale_sep3d(x64, hx, hy, hz, border=border, constant=c)
                assert_close(out.reshape(D * H, W), ref.reshape(D * H, W), sc.reshape(D * H, W), dt,
                             f"3d v{variant} {dt} r{r} {D}x{H}x{W} {border}{c}")
    finally:
        B.icl_force_variant(B.ICL_OP_CONV3D_SEP, -1)


def test_conv3d_variants_agree_bitwise_and_large_radius():
    """Every variant sums each pass in tap order with fmaf from zero, so all agree bit for bit;
    radii above the single-pass range run the three-pass variant and need the workspace."""
    D, H, W, r = 37, 45, 150, 2
    xd, _ = storage3(volume(72, D, H, W), "f32")
    hx, hy, hz = taps(72, r)
    outs = []
    for variant in range(B.icl_variant_count(B.ICL_OP_CONV3D_SEP)):
        B.check(B.icl_force_variant(B.ICL_OP_CONV3D_SEP, variant))
        try:
            outs.append(T.conv3d_sep(xd, dev(hx), dev(hy), dev(hz), workspace=ws3(D, H, W), border="constant",
                                     constant=0.25))
        finally:
            B.icl_force_variant(B.ICL_OP_CONV3D_SEP, -1)
    for o in outs[1:]:
        assert torch.equal(o.view(torch.int32), outs[0].view(torch.int32))
    r = 5
    hx, hy, hz = taps(73, r)
    xd, x64 = storage3(volume(73, 9, 12, 40), "f32")
    out = T.conv3d_sep(xd, dev(hx), dev(hy), dev(hz))
    torch.cuda.synchronize()
    assert_close(out.reshape(-1, 40), oracle.conv3d_sep(x64, hx, hy, hz).reshape(-1, 40),
                 oracle.normwise_scale_sep3d(x64, hx, hy, hz).reshape(-1, 40), "f32", "3d r5")
    o2 = torch.empty_like(xd)
    st = B.icl_conv3d_sep(xd.data_ptr(), 160, 160 * 12, o2.data_ptr(), 160, 160 * 12, 40, 12, 9, B.ICL_F32,
                          dev(hx).data_ptr(), dev(hy).data_ptr(), dev(hz).data_ptr(), r, B.ICL_BORDER_CLAMP, 0.0,
                          0, 0, torch.cuda.current_stream().cuda_stream)
    assert st == B.ICL_ERR_WORKSPACE


def test_conv3d_padded_pitches():
    """Padded rows and slices (and a misaligned start) through every variant."""
    D, H, W, r = 11, 13, 70, 2
    vol = volume(74, D, H, W)
    buf = torch.zeros(D * (H + 3) * (W + 5) + 3, dtype=torch.float32, device="cuda")
    xv = buf[1:1 + D * (H + 3) * (W + 5)].view(D, H + 3, W + 5)[:, :H, :W]
    xv.copy_(torch.from_numpy(vol).cuda())
    x64 = vol.astype(np.float64)
    hx, hy, hz = taps(74, r)
    for variant in range(B.icl_variant_count(B.ICL_OP_CONV3D_SEP)):
        B.check(B.icl_force_variant(B.ICL_OP_CONV3D_SEP, variant))
        try:
            ob = torch.full((D * (H + 1) * (W + 4),), float("nan"), dtype=torch.float32, device="cuda")
            out = ob.view(D, H + 1, W + 4)[:, :H, :W]
            T.conv3d_sep(xv, dev(hx), dev(hy), dev(hz), out=out, workspace=ws3(D, H, W))
            torch.cuda.synchronize()
            ref = oracle.conv3d_sep(x64, hx, hy, hz)
            sc = oracle.normwise_scale_sep3d(x64, hx, hy, hz)
            assert_close(out.reshape(D * H, W), ref.reshape(D * H, W), sc.reshape(D * H, W), "f32",
                         f"3d padded v{variant}")
            assert torch.isnan(ob.view(D, H + 1, W + 4)[:, H:, :]).all() and torch.isnan(
                ob.view(D, H + 1, W + 4)[:, :, W:]).all()
        finally:
            B.icl_force_variant(B.ICL_OP_CONV3D_SEP, -1)
