"""GPU parity: batched persistent separable convolution over uneven images, and its graph replay."""
import numpy as np
import pytest

from conftest import gpu_available
from helpers import assert_close, bits_of, storage, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

from oracle import oracle  # noqa: E402
from paper_1605_06399_amd import binding as B, synth  # noqa: E402

if gpu_available():
    import torch
    from paper_1605_06399_amd import torch_api as T

TORCH = {"f32": "float32", "f16": "float16", "bf16": "bfloat16"}


def make_batch(dt, count=14, lo=1, hi=300, seed=60):
    items = synth.batch_uneven(config=seed, count=count, side_lo=lo, side_hi=hi, r_lo=0, r_hi=7)
    xs, x64s, outs, taps = [], [], [], []
    for it in items:
        xd, x64 = storage(it.image, dt)
        xs.append(xd)
        x64s.append(x64)
        outs.append(torch.empty_like(xd))
        taps.append(torch.from_numpy(it.taps).cuda())
    return items, xs, x64s, outs, taps


def _nvariants(default):
    try:
        return B.icl_variant_count(B.ICL_OP_CONV_SEP_BATCHED)
    except Exception:
        return default


N_BATCHED = _nvariants(4)   # tile walks (image order, by radius, 32-row by radius), the strip walk, column walks


@pytest.fixture(params=range(N_BATCHED))
def batched_variant(request):
    if request.param >= B.icl_variant_count(B.ICL_OP_CONV_SEP_BATCHED):
        pytest.skip("no such variant")
    B.check(B.icl_force_variant(B.ICL_OP_CONV_SEP_BATCHED, request.param))
    yield request.param
    B.icl_force_variant(B.ICL_OP_CONV_SEP_BATCHED, -1)


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_batched_matches_oracle_per_image(dt, batched_variant):
    items, xs, x64s, outs, taps = make_batch(dt)
    plan = T.BatchPlan(xs, outs, taps)
    assert plan.pixels == sum(i.width * i.height for i in items)
    plan.launch()
    torch.cuda.synchronize()
    for it, x64, out, tp in zip(items, x64s, outs, taps):
        g = it.taps.astype(np.float64)
        ref = oracle.conv_sep(x64, g, g)
        assert_close(out, ref, oracle.normwise_scale_sep(x64, g, g), dt, f"batch {it.width}x{it.height} r{it.radius}")
    plan.close()


def test_batched_equals_per_image_calls(batched_variant):
    """The persistent kernels and icl_conv_sep (fused variant) agree bit for bit: every variant sums each
    output in the same tap order, whatever its tile or strip shape."""
    items, xs, _, outs, taps = make_batch("f16", count=9, seed=61)
    plan = T.BatchPlan(xs, outs, taps)
    plan.launch()
    B.check(B.icl_force_variant(B.ICL_OP_CONV_SEP, 1))
    try:
        for x, o, t in zip(xs, outs, taps):
            single = T.conv_sep(x, t, t)
            assert torch.equal(single.view(torch.int16), o.view(torch.int16))
    finally:
        B.icl_force_variant(B.ICL_OP_CONV_SEP, -1)
    plan.close()


def test_graph_replay_is_bit_identical_and_sees_new_data(batched_variant):
    items, xs, x64s, outs, taps = make_batch("bf16", count=11, seed=62)
    plan = T.BatchPlan(xs, outs, taps)
    plan.launch()
    torch.cuda.synchronize()
    eager = [bits_of(o).copy() for o in outs]
    for o in outs:
        o.fill_(0)
    for rep in range(3):                      # several replays, eager work and syncs in between
        plan.replay()
        torch.cuda.synchronize()
        for e, o in zip(eager, outs):
            assert np.array_equal(bits_of(o), e), f"replay {rep} differs"
        for o in outs:
            o.fill_(0)
        torch.cuda.synchronize()
    # taps and pixels updated in place are read by the next replay
    for t in taps:
        t.mul_(0.5)
    xs[0].copy_(xs[0] * 2)
    plan.replay()
    torch.cuda.synchronize()
    g = items[0].taps.astype(np.float64) * 0.5
    x0 = oracle.decode(bits_of(xs[0]), "bf16").reshape(xs[0].shape)
    assert_close(outs[0], oracle.conv_sep(x0, g, g), oracle.normwise_scale_sep(x0, g, g), "bf16", "after update")
    plan.close()


def test_batch_with_empty_and_tiny_images(batched_variant):
    shapes = [(0, 5), (1, 1), (3, 1), (1, 7), (70, 0), (2, 2)]
    xs, outs, taps, refs = [], [], [], []
    for k, (H, W) in enumerate(shapes):
        img = synth.image_uniform(63 + k, H, W) if H * W else np.zeros((H, W), np.float32)
        xd, x64 = storage(img, "f32")
        xs.append(xd)
        outs.append(torch.empty_like(xd))
        r = k % 4
        g = synth.gaussian_taps(r, max(r, 1) / 2)
        taps.append(torch.from_numpy(g).cuda())
        refs.append((x64, g.astype(np.float64)))
    plan = T.BatchPlan(xs, outs, taps)
    plan.launch()
    torch.cuda.synchronize()
    for (x64, g), out in zip(refs, outs):
        if x64.size:
            assert_close(out, oracle.conv_sep(x64, g, g), oracle.normwise_scale_sep(x64, g, g), "f32", "tiny")
    plan.close()
