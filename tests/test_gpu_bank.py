"""GPU parity: filter bank forward, adjoint kernels, loss and the autograd Function."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

from oracle import oracle  # noqa: E402
from paper_1605_06399_amd import binding as B, synth  # noqa: E402

if gpu_available():
    import torch
    from paper_1605_06399_amd import torch_api as T


def inputs(N, F, H, W, r, cfg=70):
    x = synth.uniform01(synth.seed(cfg, 0), N * H * W).reshape(N, 1, H, W)
    w = synth.normal(synth.seed(cfg, 1), F * (2 * r + 1) ** 2, std=0.1).reshape(F, 2 * r + 1, 2 * r + 1)
    t = synth.uniform01(synth.seed(cfg, 4), N * F * H * W).reshape(N, F, H, W)
    return x, w, t


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_normwise(got, ref, scale):
    s = np.where(scale == 0, 1.0, scale)
    return float(np.max(np.abs(got - ref) / s))


# several tiles with ragged tails, images narrower or shorter than the stencil, one row, one
# column, 1x1, and borders long enough to span several 256-pixel border segments
SHAPES = [(2, 5, 70, 133, 4), (1, 3, 64, 64, 2), (2, 2, 5, 3, 4), (1, 16, 1, 9, 1), (1, 1, 1, 1, 3), (1, 4, 65, 130, 3),
          (1, 3, 40, 1, 2), (1, 2, 2, 300, 3), (2, 2, 600, 3, 4), (1, 2, 530, 517, 1)]


def each_variant(op):
    """Run the body once per variant of `op` (forced), restoring automatic selection after."""
    for v in range(B.icl_variant_count(op)):
        B.check(B.icl_force_variant(op, v))
        try:
            yield v
        finally:
            B.icl_force_variant(op, -1)


@pytest.mark.parametrize("shape", SHAPES)
def test_bank_forward(shape):
    N, F, H, W, r = shape
    x, w, _ = inputs(N, F, H, W, r)
    ref = oracle.bank_fwd(x, w)
    scale = oracle.bank_fwd(np.abs(x), np.abs(w))
    for v in each_variant(B.ICL_OP_BANK_FWD):
        y = T.bank_fwd(cu(x), cu(w))
        torch.cuda.synchronize()
        assert rel_normwise(host(y), ref, scale) <= 1e-5, f"variant {v}"


@pytest.mark.parametrize("shape", SHAPES)
def test_bank_input_gradient(shape):
    """GPU gather (flipped correlation + edge fold) vs the oracle's scatter."""
    N, F, H, W, r = shape
    _, w, _ = inputs(N, F, H, W, r)
    gy = synth.normal(synth.seed(71, 9), N * F * H * W).reshape(N, F, H, W)
    ref = oracle.bank_bwd_input(gy, w)
    scale = oracle.bank_bwd_input(np.abs(gy), np.abs(w))
    for v in each_variant(B.ICL_OP_BANK_BWD_INPUT):
        gx = T.bank_bwd_input(cu(gy), cu(w))
        torch.cuda.synchronize()
        assert rel_normwise(host(gx), ref, scale) <= 1e-5, f"variant {v}"


@pytest.mark.parametrize("shape", SHAPES)
def test_bank_filter_gradient(shape):
    N, F, H, W, r = shape
    x, w, _ = inputs(N, F, H, W, r)
    gy = synth.normal(synth.seed(72, 9), N * F * H * W).reshape(N, F, H, W)
    ref = oracle.bank_bwd_filter(gy, x, r)
    scale = oracle.bank_bwd_filter(np.abs(gy), np.abs(x), r)
    for v in each_variant(B.ICL_OP_BANK_BWD_FILTER):
        gw = T.bank_bwd_filter(cu(gy), cu(x), r)
        torch.cuda.synchronize()
        assert rel_normwise(host(gw), ref, scale) <= 1e-5, f"variant {v}"
        # deterministic: a second call gives the same bits
        gw2 = T.bank_bwd_filter(cu(gy), cu(x), r)
        assert torch.equal(gw, gw2)


def test_bank_many_filters_falls_back():
    """More filters than the persistent kernels' tap table holds: the tiled kernels take over."""
    N, F, H, W, r = 1, 20, 33, 70, 2
    x, w, _ = inputs(N, F, H, W, r, cfg=76)
    y = T.bank_fwd(cu(x), cu(w))
    torch.cuda.synchronize()
    assert rel_normwise(host(y), oracle.bank_fwd(x, w), oracle.bank_fwd(np.abs(x), np.abs(w))) <= 1e-5


def test_sse_loss():
    y = synth.normal(synth.seed(73, 1), 1_000_003).astype(np.float32)
    t = synth.uniform01(synth.seed(73, 2), 1_000_003)
    L, gy = T.sse_loss(cu(y), cu(t))
    Lr, gyr = oracle.sse_loss(y, t)
    assert abs(L.item() - Lr) <= 1e-5 * Lr
    assert np.array_equal(host(gy), 2.0 * (y.astype(np.float32) - t).astype(np.float64))
    L2, none = T.sse_loss(cu(y), cu(t), grad=False)
    assert none is None and L2.item() == L.item()


def loss_bound(yr, t, ys, Lr):
    """|L_gpu - L| for a forward within 1e-5 * ys of yr (what test_bank_forward asserts), the float32
    subtraction y - t, and the float64 sum: sum 2|d| (1e-5 ys + 2^-23 (|y| + |t|)) + 1e-6 L."""
    return float(np.sum(2 * np.abs(yr - t) * (1e-5 * ys + 2.0 ** -23 * (np.abs(yr) + np.abs(t))))) + 1e-6 * Lr


@pytest.mark.parametrize("shape", SHAPES)
def test_bank_forward_fused_with_loss(shape):
    N, F, H, W, r = shape
    x, w, t = inputs(N, F, H, W, r)
    yr = oracle.bank_fwd(x, w)
    ys = oracle.bank_fwd(np.abs(x), np.abs(w))
    Lr, gyr = oracle.sse_loss(yr, t)
    for v in each_variant(B.ICL_OP_BANK_FWD_SSE):
        L, gy, y = T.bank_fwd_sse(cu(x), cu(w), cu(t), want_y=True)
        torch.cuda.synchronize()
        assert rel_normwise(host(y), yr, ys) <= 1e-5, f"variant {v}: y"
        assert rel_normwise(host(gy), gyr, 2 * ys + 2 * np.abs(t)) <= 1e-5, f"variant {v}: gy"
        assert abs(L.item() - Lr) <= loss_bound(yr, t, ys, Lr), f"variant {v}: L {L.item()} vs {Lr}"
        # the optional outputs change nothing else: same loss bits, same gradient bits
        L2, gy2, none = T.bank_fwd_sse(cu(x), cu(w), cu(t))
        L3, none2, _ = T.bank_fwd_sse(cu(x), cu(w), cu(t), grad=False)
        assert none is None and none2 is None
        assert L2.item() == L.item() == L3.item()
        assert torch.equal(gy2, gy)


@pytest.mark.parametrize("shape", [(2, 5, 70, 133, 4), (1, 16, 64, 64, 2), (1, 3, 33, 70, 3), (2, 2, 5, 3, 1)])
def test_fused_outputs_equal_forward_then_loss(shape):
    """A fused variant sums the taps in the same order as the forward variant of its family
    (the FMA variants all alike, the matrix-core variant its own way), so its y and gy are
    the same bits as that forward followed by icl_sse_loss."""
    N, F, H, W, r = shape
    x, w, t = inputs(N, F, H, W, r, cfg=77)
    xt, wt, tt = cu(x), cu(w), cu(t)
    fwd_names = B.variant_names(B.ICL_OP_BANK_FWD)
    refs = {}
    for fam in ("pers_p4x4", "mfma_t64"):
        B.check(B.icl_force_variant(B.ICL_OP_BANK_FWD, fwd_names.index(fam)))
        try:
            y_ref = T.bank_fwd(xt, wt)
        finally:
            B.icl_force_variant(B.ICL_OP_BANK_FWD, -1)
        refs[fam] = (y_ref, T.sse_loss(y_ref, tt)[1])
    sse_names = B.variant_names(B.ICL_OP_BANK_FWD_SSE)
    for v in each_variant(B.ICL_OP_BANK_FWD_SSE):
        _, gy, y = T.bank_fwd_sse(xt, wt, tt, want_y=True)
        y_ref, gy_ref = refs["mfma_t64" if sse_names[v].startswith("mfma") else "pers_p4x4"]
        assert torch.equal(y, y_ref), f"variant {v}: y"
        assert torch.equal(gy, gy_ref), f"variant {v}: gy"


def test_fused_loss_many_filters_and_empty():
    N, F, H, W, r = 1, 20, 33, 70, 2          # beyond the persistent kernel's tap table: plain variant
    x, w, t = inputs(N, F, H, W, r, cfg=78)
    yr = oracle.bank_fwd(x, w)
    Lr, _ = oracle.sse_loss(yr, t)
    L, gy, _ = T.bank_fwd_sse(cu(x), cu(w), cu(t))
    torch.cuda.synchronize()
    assert abs(L.item() - Lr) <= loss_bound(yr, t, oracle.bank_fwd(np.abs(x), np.abs(w)), Lr)
    e = torch.empty((0, 1, 8, 8), dtype=torch.float32, device="cuda")
    L0, gy0, _ = T.bank_fwd_sse(e, cu(w), torch.empty((0, F, 8, 8), dtype=torch.float32, device="cuda"))
    assert L0.item() == 0.0 and gy0.numel() == 0


def test_loss_function_backward_matches_oracle_chain():
    """filter_bank_loss(x, w, t).backward(): fused forward, saved gy, the two adjoint kernels."""
    N, F, H, W, r = 2, 6, 40, 57, 4
    x, w, t = inputs(N, F, H, W, r, cfg=79)
    xt = cu(x).requires_grad_(True)
    wt = cu(w).requires_grad_(True)
    L = T.filter_bank_loss(xt, wt, cu(t))
    L.backward()
    torch.cuda.synchronize()
    yr = oracle.bank_fwd(x, w)
    Lr, gyr = oracle.sse_loss(yr, t)
    ys = oracle.bank_fwd(np.abs(x), np.abs(w))
    assert abs(L.item() - Lr) <= loss_bound(yr, t, ys, Lr)
    gxr = oracle.bank_bwd_input(gyr, w)
    gwr = oracle.bank_bwd_filter(gyr, x, r)
    sx = oracle.bank_bwd_input(np.abs(gyr), np.abs(w)) + 2 * oracle.bank_bwd_input(ys, np.abs(w))
    sw = oracle.bank_bwd_filter(np.abs(gyr), np.abs(x), r) + 2 * oracle.bank_bwd_filter(ys, np.abs(x), r)
    assert rel_normwise(host(xt.grad), gxr, sx) <= 1e-5
    assert rel_normwise(host(wt.grad), gwr, sw) <= 1e-5
    # an upstream factor scales both gradients inside the adjoint kernels: each output is the
    # float32 product of the unscaled sum and the factor, rounded once (bit for bit on the host)
    gx1 = xt.grad.detach().clone()
    gw1 = wt.grad.detach().clone()
    xt.grad = None
    wt.grad = None
    (3.0 * T.filter_bank_loss(xt, wt, cu(t))).backward()
    assert rel_normwise(host(xt.grad), 3 * gxr, 3 * sx) <= 1e-5
    three = np.float32(3.0)
    assert np.array_equal(xt.grad.cpu().numpy(), gx1.cpu().numpy() * three)
    assert np.array_equal(wt.grad.cpu().numpy(), gw1.cpu().numpy() * three)


@pytest.mark.parametrize("shape", SHAPES[:6])
def test_adjoint_output_factor_every_variant(shape):
    """The `scale` argument of both adjoints multiplies each output once: with a factor of one the
    result equals the call without it bit for bit, and with -0.75 it equals the float32 product of
    that result and the factor, for every variant."""
    N, F, H, W, r = shape
    x, w, _ = inputs(N, F, H, W, r, cfg=81)
    gy = synth.uniform01(synth.seed(81, 6), N * F * H * W).reshape(N, F, H, W) * 2 - 1
    gyt, wt, xt = cu(gy), cu(w), cu(x)
    one = torch.ones(1, dtype=torch.float32, device="cuda")
    fac = torch.full((1,), -0.75, dtype=torch.float32, device="cuda")
    for _ in each_variant(B.ICL_OP_BANK_BWD_INPUT):
        g0 = T.bank_bwd_input(gyt, wt)
        assert torch.equal(T.bank_bwd_input(gyt, wt, scale=one), g0)
        g1 = T.bank_bwd_input(gyt, wt, scale=fac)
        assert np.array_equal(g1.cpu().numpy(), g0.cpu().numpy() * np.float32(-0.75))
    for _ in each_variant(B.ICL_OP_BANK_BWD_FILTER):
        w0 = T.bank_bwd_filter(gyt, xt, r)
        assert torch.equal(T.bank_bwd_filter(gyt, xt, r, scale=one), w0)
        w1 = T.bank_bwd_filter(gyt, xt, r, scale=fac)
        assert np.array_equal(w1.cpu().numpy(), w0.cpu().numpy() * np.float32(-0.75))


def test_autograd_function_matches_oracle_chain():
    """loss.backward() through FilterBankFn vs the oracle's forward -> loss -> adjoints (same x, w, t)."""
    N, F, H, W, r = 2, 6, 40, 57, 4
    x, w, t = inputs(N, F, H, W, r, cfg=74)
    xt = cu(x).requires_grad_(True)
    wt = cu(w).requires_grad_(True)
    y = T.filter_bank(xt, wt)
    L, gy = T.sse_loss(y.detach(), cu(t))
    y.backward(gy)
    torch.cuda.synchronize()
    yr = oracle.bank_fwd(x, w)
    Lr, gyr = oracle.sse_loss(yr, t)
    gxr = oracle.bank_bwd_input(gyr, w)
    gwr = oracle.bank_bwd_filter(gyr, x, r)
    assert abs(L.item() - Lr) <= 1e-5 * Lr
    sx = oracle.bank_bwd_input(np.abs(gyr), np.abs(w))
    sw = oracle.bank_bwd_filter(np.abs(gyr), np.abs(x), r)
    # gy carries the forward's float32 error (<= 1e-5 normwise), amplified by at most the stencil sums
    assert rel_normwise(host(xt.grad), gxr, sx + 2 * oracle.bank_bwd_input(oracle.bank_fwd(np.abs(x), np.abs(w)), np.abs(w))) <= 1e-5
    assert rel_normwise(host(wt.grad), gwr, sw + 2 * oracle.bank_bwd_filter(oracle.bank_fwd(np.abs(x), np.abs(w)), np.abs(x), r)) <= 1e-5


def test_gpu_gradient_against_float32_central_differences():
    """Central differences of the GPU loss (eps 1e-3) on a tiny problem.  The loss is quadratic, so
    the difference quotient is exact up to float32 cancellation (~ulp(L)/eps), hence rtol 2e-2."""
    N, F, H, W, r = 1, 2, 9, 7, 2
    x, w, t = inputs(N, F, H, W, r, cfg=75)
    xt, wt, tt = cu(x), cu(w), cu(t)

    def loss(xx, ww):
        return T.sse_loss(T.bank_fwd(xx, ww), tt, grad=False)[0].item()

    y = T.bank_fwd(xt, wt)
    _, gy = T.sse_loss(y, tt)
    gx = host(T.bank_bwd_input(gy, wt))
    gw = host(T.bank_bwd_filter(gy, xt, r))
    eps = 1e-3
    for (yy, xx) in [(0, 0), (8, 6), (4, 3), (0, 5)]:
        xp, xm = xt.clone(), xt.clone()
        xp[0, 0, yy, xx] += eps
        xm[0, 0, yy, xx] -= eps
        fd = (loss(xp, wt) - loss(xm, wt)) / (2 * eps)
        assert fd == pytest.approx(gx[0, 0, yy, xx], rel=2e-2, abs=2e-2)
    for idx in [(0, 0, 0), (1, 2, 2), (0, 4, 1)]:
        wp, wm = wt.clone(), wt.clone()
        wp[idx] += eps
        wm[idx] -= eps
        fd = (loss(xt, wp) - loss(xt, wm)) / (2 * eps)
        assert fd == pytest.approx(gw[idx], rel=2e-2, abs=2e-2)
