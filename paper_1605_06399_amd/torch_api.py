"""torch-tensor front end of the C ABI.

PyTorch supplies device memory and the current HIP stream; each function here
checks devices, dtypes and strides, derives pitches in bytes and calls the
library.  Nothing is computed in torch: outputs are allocated with
``torch.empty`` and filled by the HIP kernels.
"""
from __future__ import annotations

import torch

from . import binding as B

_DT = {torch.float32: B.ICL_F32, torch.float16: B.ICL_F16, torch.bfloat16: B.ICL_BF16}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _image(t: torch.Tensor, name: str):
    """(pointer, pitch_bytes, width, height, icl dtype) of a 2-D row-major image view."""
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D (H, W)")
    es = t.element_size()
    if t.numel() == 0:
        return 0, t.shape[1] * es, t.shape[1], t.shape[0]
    if t.stride(1) != 1 and t.shape[1] > 1:
        raise ValueError(f"{name} rows must be contiguous (stride(1) == 1)")
    pitch = t.stride(0) * es if t.shape[0] > 1 else t.shape[1] * es
    return t.data_ptr(), pitch, t.shape[1], t.shape[0]


def _taps(t: torch.Tensor, n: int, name: str) -> int:
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous float32 GPU tensor with {n} taps")
    return t.data_ptr()


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 4) // 4 + 1, dtype=torch.float32, device=device)


_BORDERS = {"clamp": B.ICL_BORDER_CLAMP, "constant": B.ICL_BORDER_CONSTANT}


def _border(border: str) -> int:
    if border not in _BORDERS:
        raise ValueError(f"border must be one of {sorted(_BORDERS)}")
    return _BORDERS[border]


def conv_sep(x: torch.Tensor, taps_x: torch.Tensor, taps_y: torch.Tensor, out: torch.Tensor | None = None,
             workspace: torch.Tensor | None = None, border: str = "clamp", constant: float = 0.0) -> torch.Tensor:
    r = (taps_x.numel() - 1) // 2
    if out is None:
        out = torch.empty_like(x, memory_format=torch.contiguous_format)
    sp, spitch, W, H = _image(x, "x")
    dp, dpitch, _, _ = _image(out, "out")
    dt = _DT[x.dtype]
    if workspace is None and r > 7:
        _, nb = B.icl_workspace_size(B.ICL_OP_CONV_SEP, W, H, dtype=dt)
        workspace = _workspace(nb, x.device)
    ws, wsb = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None else (0, 0)
    tx, ty = _taps(taps_x, 2 * r + 1, "taps_x"), _taps(taps_y, 2 * r + 1, "taps_y")
    if border == "clamp":
        B.check(B.icl_conv_sep(sp, spitch, dp, dpitch, W, H, dt, tx, ty, r, ws, wsb, _stream()), "icl_conv_sep")
    else:
        B.check(B.icl_conv_sep_border(sp, spitch, dp, dpitch, W, H, dt, tx, ty, r, _border(border), float(constant),
                                      ws, wsb, _stream()), "icl_conv_sep_border")
    return out


def conv2d(x: torch.Tensor, taps: torch.Tensor, out: torch.Tensor | None = None, border: str = "clamp",
           constant: float = 0.0) -> torch.Tensor:
    n = taps.shape[-1]
    r = (n - 1) // 2
    if out is None:
        out = torch.empty_like(x, memory_format=torch.contiguous_format)
    sp, spitch, W, H = _image(x, "x")
    dp, dpitch, _, _ = _image(out, "out")
    tp = _taps(taps, n * n, "taps")
    if border == "clamp":
        B.check(B.icl_conv2d(sp, spitch, dp, dpitch, W, H, _DT[x.dtype], tp, r, _stream()), "icl_conv2d")
    else:
        B.check(B.icl_conv2d_border(sp, spitch, dp, dpitch, W, H, _DT[x.dtype], tp, r, _border(border),
                                    float(constant), _stream()), "icl_conv2d_border")
    return out


def _volume(t: torch.Tensor, name: str):
    """(pointer, row pitch, slice pitch, W, H, D) of a 3-D [D, H, W] view with contiguous rows."""
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dim() != 3:
        raise ValueError(f"{name} must be 3-D (D, H, W)")
    es = t.element_size()
    D, H, W = t.shape
    if t.numel() == 0:
        return 0, W * es, H * W * es, W, H, D
    if t.stride(2) != 1 and W > 1:
        raise ValueError(f"{name} rows must be contiguous (stride(2) == 1)")
    rp = t.stride(1) * es if H > 1 else W * es
    sp = t.stride(0) * es if D > 1 else (H - 1) * rp + W * es
    return t.data_ptr(), rp, sp, W, H, D


def conv3d_sep(x: torch.Tensor, taps_x: torch.Tensor, taps_y: torch.Tensor, taps_z: torch.Tensor,
               out: torch.Tensor | None = None, workspace: torch.Tensor | None = None, border: str = "clamp",
               constant: float = 0.0) -> torch.Tensor:
    """Separable 3-D correlation of a [D, H, W] volume."""
    r = (taps_x.numel() - 1) // 2
    if out is None:
        out = torch.empty_like(x, memory_format=torch.contiguous_format)
    sp, srp, ssp, W, H, D = _volume(x, "x")
    dp, drp, dsp, _, _, _ = _volume(out, "out")
    dt = _DT[x.dtype]
    if workspace is None and r > 3:
        _, nb = B.icl_workspace_size(B.ICL_OP_CONV3D_SEP, W, H, n=D, dtype=dt)
        workspace = _workspace(nb, x.device)
    ws, wsb = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None else (0, 0)
    n = 2 * r + 1
    B.check(B.icl_conv3d_sep(sp, srp, ssp, dp, drp, dsp, W, H, D, dt, _taps(taps_x, n, "taps_x"),
                             _taps(taps_y, n, "taps_y"), _taps(taps_z, n, "taps_z"), r, _border(border),
                             float(constant), ws, wsb, _stream()), "icl_conv3d_sep")
    return out


def conv2d_u8(x: torch.Tensor, taps: torch.Tensor, shift: int, out: torch.Tensor | None = None,
              border: str = "clamp", constant: int = 0) -> torch.Tensor:
    """unsigned char image, int16 taps [(2r+1), (2r+1)]: exact integer sum, rounded shift, saturated."""
    if x.dtype != torch.uint8:
        raise ValueError("x must be a uint8 image")
    n = taps.shape[-1]
    r = (n - 1) // 2
    if not taps.is_cuda or taps.dtype != torch.int16 or not taps.is_contiguous() or taps.numel() != n * n:
        raise ValueError(f"taps must be a contiguous int16 GPU tensor with {n * n} values")
    if out is None:
        out = torch.empty_like(x, memory_format=torch.contiguous_format)
    if out.dtype != torch.uint8:
        raise ValueError("out must be a uint8 image")
    sp, spitch, W, H = _image(x, "x")
    dp, dpitch, _, _ = _image(out, "out")
    B.check(B.icl_conv2d_u8(sp, spitch, dp, dpitch, W, H, taps.data_ptr(), r, int(shift), _border(border),
                            int(constant), _stream()), "icl_conv2d_u8")
    return out


def harris(x: torch.Tensor, window_taps: torch.Tensor, k: float = 0.04, out: torch.Tensor | None = None,
           workspace: torch.Tensor | None = None) -> torch.Tensor:
    if x.dtype != torch.float32:
        raise ValueError("harris takes a float32 image")
    rg = (window_taps.numel() - 1) // 2
    if out is None:
        out = torch.empty_like(x, memory_format=torch.contiguous_format)
    sp, spitch, W, H = _image(x, "x")
    dp, dpitch, _, _ = _image(out, "out")
    if workspace is None and rg > 3:
        _, nb = B.icl_workspace_size(B.ICL_OP_HARRIS, W, H)
        workspace = _workspace(nb, x.device)
    ws, wsb = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None else (0, 0)
    B.check(B.icl_harris(sp, spitch, dp, dpitch, W, H, _taps(window_taps, 2 * rg + 1, "window_taps"), rg, float(k),
                         ws, wsb, _stream()), "icl_harris")
    return out


def nms(resp: torch.Tensor, threshold: float, radius: int = 1, out: torch.Tensor | None = None) -> torch.Tensor:
    if resp.dtype != torch.float32:
        raise ValueError("nms takes a float32 response")
    if out is None:
        out = torch.empty(resp.shape, dtype=torch.uint8, device=resp.device)
    sp, spitch, W, H = _image(resp, "resp")
    dp, dpitch, _, _ = _image(out, "out")
    B.check(B.icl_nms(sp, spitch, dp, dpitch, W, H, int(radius), float(threshold), _stream()), "icl_nms")
    return out


def corners(x: torch.Tensor, window_taps: torch.Tensor, k: float = 0.04, threshold: float = 1e-3,
            nms_radius: int = 1, out: torch.Tensor | None = None, resp: torch.Tensor | None = None,
            workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Harris response and non-maximum suppression in one call: the uint8 corner mask.  Pass a
    float32 `resp` image to also receive the response."""
    if x.dtype != torch.float32:
        raise ValueError("x must be float32")
    r = (window_taps.numel() - 1) // 2
    if out is None:
        out = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    sp, spitch, W, H = _image(x, "x")
    mp, mpitch, _, _ = _image(out, "out")
    rp, rpitch = (0, 0)
    if resp is not None:
        if resp.dtype != torch.float32:
            raise ValueError("resp must be float32")
        rp, rpitch, _, _ = _image(resp, "resp")
    ws, wsb = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None else (0, 0)
    B.check(B.icl_corners(sp, spitch, mp, mpitch, W, H, _taps(window_taps, 2 * r + 1, "window_taps"), r, float(k),
                          int(nms_radius), float(threshold), rp, rpitch, ws, wsb, _stream()), "icl_corners")
    return out


def tune(op: int, dtype: torch.dtype, radius: int, width: int, height: int) -> None:
    B.check(B.icl_tune(op, _DT[dtype], radius, width, height, _stream()), "icl_tune")


# ----------------------------------------------------------------------------- batched

class BatchPlan:
    """Tile table for a batch of uneven images, launched as one persistent kernel.

    ``images`` / ``outputs`` are 2-D GPU tensors of one dtype; ``taps`` are float32
    GPU tensors (2r+1), used for both passes of each image.  The plan keeps
    references to all of them, so the pointers it uploaded stay valid.
    """

    def __init__(self, images, outputs, taps_x, taps_y=None):
        taps_y = taps_x if taps_y is None else taps_y
        self._keep = (list(images), list(outputs), list(taps_x), list(taps_y))
        dts = {t.dtype for t in images} | {t.dtype for t in outputs}
        if len(dts) != 1:
            raise ValueError("all images and outputs must share one dtype")
        self.dtype = dts.pop()
        descs = []
        for x, y, tx, ty in zip(*self._keep):
            sp, spitch, W, H = _image(x, "image")
            dp, dpitch, W2, H2 = _image(y, "output")
            if (W, H) != (W2, H2):
                raise ValueError("output shape differs from its image")
            r = (tx.numel() - 1) // 2
            descs.append(B.icl_image_desc(sp, dp, spitch, dpitch, W, H, r, _taps(tx, 2 * r + 1, "taps_x"),
                                          _taps(ty, 2 * r + 1, "taps_y")))
        st, self.handle = B.icl_batch_plan_create(descs, _DT[self.dtype])
        B.check(st, "icl_batch_plan_create")
        _, self.tiles, self.pixels = B.icl_batch_plan_info(self.handle)
        self._graph = None

    def launch(self) -> None:
        B.check(B.icl_conv_sep_batched(self.handle, _stream()), "icl_conv_sep_batched")

    def tune(self) -> None:
        """Per-device choice of the walk for this plan (writes the outputs; a graph made before
        keeps the walk it captured, so tune first)."""
        B.check(B.icl_batch_plan_tune(self.handle, _stream()), "icl_batch_plan_tune")

    def variant(self) -> int:
        st, v = B.icl_batch_plan_variant(self.handle)
        B.check(st, "icl_batch_plan_variant")
        return v

    def graph(self):
        """hipGraphExec holding the single persistent launch (created once)."""
        if self._graph is None:
            st, g = B.icl_batch_graph_create(self.handle)
            B.check(st, "icl_batch_graph_create")
            self._graph = g
        return self._graph

    def replay(self) -> None:
        B.check(B.icl_graph_launch(self.graph(), _stream()), "icl_graph_launch")

    def close(self) -> None:
        if self._graph is not None:
            B.icl_graph_destroy(self._graph)
            self._graph = None
        if self.handle:
            B.icl_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- filter bank

def _dense(t: torch.Tensor, name: str, dtype=torch.float32) -> int:
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} GPU tensor")
    return t.data_ptr()


def bank_fwd(x: torch.Tensor, w: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    N, H, W = x.shape[0], x.shape[-2], x.shape[-1]
    F, r = w.shape[0], (w.shape[-1] - 1) // 2
    if out is None:
        out = torch.empty((N, F, H, W), dtype=torch.float32, device=x.device)
    B.check(B.icl_bank_fwd(_dense(x, "x"), _dense(w, "w"), _dense(out, "y"), N, F, H, W, r, _stream()),
            "icl_bank_fwd")
    return out


def _scale(scale: torch.Tensor | None) -> int:
    """Device address of a float32 scalar output factor (0: none)."""
    if scale is None:
        return 0
    if scale.numel() != 1 or scale.dtype != torch.float32 or not scale.is_cuda:
        raise ValueError("scale must be a one-element float32 GPU tensor")
    return scale.data_ptr()


def bank_bwd_input(gy: torch.Tensor, w: torch.Tensor, out: torch.Tensor | None = None,
                   scale: torch.Tensor | None = None) -> torch.Tensor:
    N, F, H, W = gy.shape
    r = (w.shape[-1] - 1) // 2
    if out is None:
        out = torch.empty((N, 1, H, W), dtype=torch.float32, device=gy.device)
    B.check(B.icl_bank_bwd_input(_dense(gy, "gy"), _dense(w, "w"), _dense(out, "gx"), N, F, H, W, r, _stream(),
                                 scale=_scale(scale)), "icl_bank_bwd_input")
    return out


def bank_bwd_filter(gy: torch.Tensor, x: torch.Tensor, radius: int, out: torch.Tensor | None = None,
                    workspace: torch.Tensor | None = None, scale: torch.Tensor | None = None) -> torch.Tensor:
    N, F, H, W = gy.shape
    k = 2 * radius + 1
    if out is None:
        out = torch.empty((F, k, k), dtype=torch.float32, device=gy.device)
    if workspace is None:
        _, nb = B.icl_workspace_size(B.ICL_OP_BANK_BWD_FILTER, W, H, N, F, radius)
        workspace = _workspace(nb, gy.device)
    B.check(B.icl_bank_bwd_filter(_dense(gy, "gy"), _dense(x, "x"), _dense(out, "gw"), N, F, H, W, radius,
                                  workspace.data_ptr(), workspace.numel() * 4, _stream(), scale=_scale(scale)),
            "icl_bank_bwd_filter")
    return out


def sse_loss(y: torch.Tensor, t: torch.Tensor, grad: bool = True, workspace: torch.Tensor | None = None):
    """(L, gy): L = sum (y - t)^2 as a 0-d GPU tensor, gy = 2 (y - t) (None if grad is False)."""
    if y.shape != t.shape:
        raise ValueError("y and t differ in shape")
    loss = torch.empty((), dtype=torch.float32, device=y.device)
    gy = torch.empty_like(y) if grad else None
    if workspace is None:
        _, nb = B.icl_workspace_size(B.ICL_OP_SSE_LOSS, y.numel(), 1)
        workspace = _workspace(nb, y.device)
    B.check(B.icl_sse_loss(_dense(y, "y"), _dense(t, "t"), gy.data_ptr() if gy is not None else 0, y.numel(),
                           loss.data_ptr(), workspace.data_ptr(), workspace.numel() * 4, _stream()), "icl_sse_loss")
    return loss, gy


def bank_fwd_sse(x: torch.Tensor, w: torch.Tensor, t: torch.Tensor, grad: bool = True, want_y: bool = False,
                 workspace: torch.Tensor | None = None, gy: torch.Tensor | None = None,
                 y: torch.Tensor | None = None):
    """Forward fused with the loss: (L, gy, y) with L = sum (bank(x, w) - t)^2 as a 0-d GPU tensor,
    gy = 2 (bank(x, w) - t) (None if grad is False) and the forward output y (None unless want_y)."""
    N, H, W = x.shape[0], x.shape[-2], x.shape[-1]
    F, r = w.shape[0], (w.shape[-1] - 1) // 2
    if tuple(t.shape) != (N, F, H, W):
        raise ValueError(f"target shape {tuple(t.shape)} != {(N, F, H, W)}")
    loss = torch.empty((), dtype=torch.float32, device=x.device)
    if grad and gy is None:
        gy = torch.empty((N, F, H, W), dtype=torch.float32, device=x.device)
    if want_y and y is None:
        y = torch.empty((N, F, H, W), dtype=torch.float32, device=x.device)
    gy = gy if grad else None
    y = y if want_y else None
    if workspace is None:
        _, nb = B.icl_workspace_size(B.ICL_OP_BANK_FWD_SSE, W, H, N, F, r)
        workspace = _workspace(nb, x.device)
    B.check(B.icl_bank_fwd_sse(_dense(x, "x"), _dense(w, "w"), _dense(t, "t"),
                               _dense(y, "y") if y is not None else 0, _dense(gy, "gy") if gy is not None else 0,
                               loss.data_ptr(), N, F, H, W, r, workspace.data_ptr(), workspace.numel() * 4,
                               _stream()), "icl_bank_fwd_sse")
    return loss, gy, y


class FilterBankFn(torch.autograd.Function):
    """y = bank(x, w) with hand-written adjoint kernels for both gradients."""

    @staticmethod
    def forward(ctx, x, w):
        ctx.save_for_backward(x, w)
        return bank_fwd(x.contiguous(), w.contiguous())

    @staticmethod
    def backward(ctx, gy):
        x, w = ctx.saved_tensors
        gy = gy.contiguous()
        gx = bank_bwd_input(gy, w.contiguous()).view_as(x) if ctx.needs_input_grad[0] else None
        gw = bank_bwd_filter(gy, x.contiguous(), (w.shape[-1] - 1) // 2) if ctx.needs_input_grad[1] else None
        return gx, gw


def filter_bank(x: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    return FilterBankFn.apply(x, w)


class FilterBankLossFn(torch.autograd.Function):
    """L = sum (bank(x, w) - t)^2 from the fused forward (y is never stored); the backward runs
    the two adjoint kernels on the saved gy = 2 (y - t).  The target is a constant (no gradient)."""

    @staticmethod
    def forward(ctx, x, w, t):
        L, gy, _ = bank_fwd_sse(x.contiguous(), w.contiguous(), t.contiguous())
        ctx.save_for_backward(x, w, gy)
        return L

    @staticmethod
    def backward(ctx, gL):
        x, w, gy = ctx.saved_tensors
        # chain rule for the upstream factor on L (1 for loss.backward()): the adjoint kernels take
        # it as their output factor (read on the device, so no host synchronisation)
        sc = gL.detach().to(device=gy.device, dtype=torch.float32).reshape(1).contiguous()
        gx = bank_bwd_input(gy, w.contiguous(), scale=sc).view_as(x) if ctx.needs_input_grad[0] else None
        gw = bank_bwd_filter(gy, x.contiguous(), (w.shape[-1] - 1) // 2, scale=sc) if ctx.needs_input_grad[1] else None
        return gx, gw, None


def filter_bank_loss(x: torch.Tensor, w: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
    return FilterBankLossFn.apply(x, w, t)
