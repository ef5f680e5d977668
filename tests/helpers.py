"""Shared test helpers: device tensors, padded views and the tolerance rules.

Tolerances (stated per result):
  float32 storage : normwise error |y_gpu - y| / S <= 1e-5, where S is the same
                    stencil evaluated on absolute values (|taps|, |input|) by the
                    oracle; S == 0 requires exact equality.
  float16 storage : normwise error against the FP64 oracle <= 2e-3 (binary16's
                    half-ulp is 4.9e-4 relative, so the budget covers one output
                    rounding plus float32 accumulation).
  Harris response : |R_gpu - R| <= D(p), the oracle's bound on the rounding error of any
                    float32 evaluation order of the chain (Sobel, products, window,
                    response; oracle.harris_f32_bound).  The same D decides which
                    corner-mask pixels rounding may flip (nms_ambiguous).
  bfloat16 storage: |y_gpu - y| <= ulp_bf16(y) + 1e-5 * S: at most one bfloat16
                    ulp of output rounding on top of the float32 accumulation
                    budget.  (bfloat16's own half-ulp, up to 2^-8 = 3.9e-3
                    relative, exceeds 2e-3, so the 2e-3 figure cannot bind it;
                    near-zero outputs of cancelling sums need the S term.)  The
                    normwise error against FP64 is returned alongside.
"""
from __future__ import annotations

import numpy as np

try:
    import torch
except Exception:  # pragma: no cover
    torch = None

from paper_1605_06399_amd import synth

TORCH_DT = {"f32": "float32", "f16": "float16", "bf16": "bfloat16"}


def dev():
    return torch.device("cuda:0")


def storage(img_f32: np.ndarray, dt: str):
    """(device tensor in the storage dtype, float64 values the oracle must see)."""
    from oracle import oracle
    if dt == "f32":
        t = torch.from_numpy(np.ascontiguousarray(img_f32, dtype=np.float32)).to(dev())
        return t, img_f32.astype(np.float64)
    if dt == "f16":
        bits = synth.to_f16_bits(img_f32)
        t = torch.from_numpy(bits.view(np.int16).copy()).to(dev()).view(torch.float16)
        return t, oracle.decode(bits, "f16")
    bits = synth.to_bf16_bits(img_f32)
    t = torch.from_numpy(bits.view(np.int16).copy()).to(dev()).view(torch.bfloat16)
    return t, oracle.decode(bits, "bf16")


def padded_view(t, pad_elems: int, offset_elems: int = 0):
    """Copy of a 2-D tensor inside a larger buffer: row pitch W + pad, start offset."""
    H, W = t.shape
    buf = torch.zeros((H + 1) * (W + pad_elems) + offset_elems + 16, dtype=t.dtype, device=t.device)
    v = buf[offset_elems:offset_elems + H * (W + pad_elems)].view(H, W + pad_elems)[:, :W]
    v.copy_(t)
    return v


def empty_padded(H, W, dtype, pad_elems: int, offset_elems: int = 0):
    buf = torch.full(((H + 1) * (W + pad_elems) + offset_elems + 16,), float("nan"), dtype=dtype, device=dev())
    return buf[offset_elems:offset_elems + H * (W + pad_elems)].view(H, W + pad_elems)[:, :W]


def to_host(t) -> np.ndarray:
    """Device image -> float64 (bf16/f16 decoded by numpy/torch on the host)."""
    return t.detach().float().cpu().numpy().astype(np.float64)


def bits_of(t) -> np.ndarray:
    return t.detach().contiguous().view(torch.int16).cpu().numpy().view(np.uint16)


def normwise(got: np.ndarray, ref: np.ndarray, scale: np.ndarray) -> float:
    d = np.abs(got - ref)
    zero = scale == 0
    if np.any(d[zero] != 0):
        return float("inf")
    s = np.where(zero, 1.0, scale)
    return float(np.max(d / s)) if d.size else 0.0


def assert_close(out, ref64: np.ndarray, scale: np.ndarray, dt: str, what: str = ""):
    """Apply the stated tolerance of the storage type (see module docstring)."""
    from oracle import oracle
    got = to_host(out)
    err = normwise(got, ref64, scale)
    if dt == "f32":
        assert err <= 1e-5, f"{what}: float32 normwise error {err:.3e} > 1e-5"
    elif dt == "f16":
        assert err <= 2e-3, f"{what}: float16 normwise error {err:.3e} > 2e-3"
    else:
        bad = bf16_violations(got, ref64, scale)
        assert bad == 0, f"{what}: {bad} bfloat16 outputs beyond 1 ulp + 1e-5 S (normwise {err:.3e})"
    return err


def ulp_bf16(y: np.ndarray) -> np.ndarray:
    """Spacing of bfloat16 numbers at |y| (8 significant bits; subnormal spacing 2^-133)."""
    a = np.abs(y)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, np.ldexp(1.0, (np.maximum(e, -126) - 7).astype(np.int64)), 2.0 ** -133)


def bf16_violations(got: np.ndarray, ref64: np.ndarray, scale: np.ndarray) -> int:
    return int(np.sum(np.abs(got - ref64) > ulp_bf16(ref64) + 1e-5 * scale))


def nms_ambiguous(R: np.ndarray, D: np.ndarray, tau: float, radius: int = 1) -> np.ndarray:
    """Pixels whose 3x3 (or (2r+1)^2) NMS decision float32 rounding of the response may flip:
    |R - tau| <= D(p), or |R(p) - R(q)| <= D(p) + D(q) for a clamped neighbour q other than p
    itself (a neighbour clamped onto p compares R(p) >= R(p), which no rounding changes).
    Elsewhere the mask of a response within D of R equals the mask of R."""
    H, W = R.shape
    amb = np.abs(R - tau) <= D
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            if dx == 0 and dy == 0:
                continue
            yy = np.clip(np.arange(H)[:, None] + dy, 0, H - 1)
            xx = np.clip(np.arange(W)[None, :] + dx, 0, W - 1)
            other = (yy != np.arange(H)[:, None]) | (xx != np.arange(W)[None, :])
            amb |= other & (np.abs(R - R[yy, xx]) <= D + D[yy, xx])
    return amb
