"""torch.autograd.Function over the differentiable batch of the C ABI.

forward: eapdtw_dtw_fwd (plain DTW of each pair, band checkpoints kept);
backward: eapdtw_dtw_bwd (tile-wise recomputation from the checkpoints,
backtracking of the optimal warping path, scatter of 2(S(i)-T(j)) * g onto
both inputs).  Section 2: DTW is the cost of the optimal warping path, so its
gradient is the gradient of that path's cost.
"""
from __future__ import annotations

import ctypes

import torch


class DTWFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, S: torch.Tensor, T: torch.Tensor, window: int):
        from . import _dev, _ptr, context
        S32, T32 = _dev(S), _dev(T)
        if S32.shape != T32.shape or S32.dim() != 2:
            raise ValueError("S and T must both be [npairs, len]")
        P, L = S32.shape
        c = context(S32.device.index)
        c.bind_stream()
        nbytes = c._lib.eapdtw_dtw_ckpt_bytes(P, L, int(window))
        if nbytes < 0:
            raise ValueError("unsupported sizes for the differentiable batch")
        ckpt = torch.empty(max(int(nbytes), 1), device=S32.device, dtype=torch.uint8)
        out = torch.empty(P, device=S32.device, dtype=torch.float32)
        c.check(c._lib.eapdtw_dtw_fwd(c.handle, _ptr(S32), _ptr(T32), P, L, int(window), _ptr(out),
                                      ctypes.c_void_p(ckpt.data_ptr())))
        ctx.save_for_backward(S32, T32, ckpt)
        ctx.window = int(window)
        ctx.in_dtypes = (S.dtype, T.dtype)
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        from . import _ptr, context
        S32, T32, ckpt = ctx.saved_tensors
        P, L = S32.shape
        g = grad_out.to(torch.float32).contiguous()
        c = context(S32.device.index)
        c.bind_stream()
        gS = torch.empty_like(S32)
        gT = torch.empty_like(T32)
        c.check(c._lib.eapdtw_dtw_bwd(c.handle, _ptr(S32), _ptr(T32), P, L, ctx.window,
                                      ctypes.c_void_p(ckpt.data_ptr()), _ptr(g), _ptr(gS),
                                      _ptr(gT)))
        return gS.to(ctx.in_dtypes[0]), gT.to(ctx.in_dtypes[1]), None
