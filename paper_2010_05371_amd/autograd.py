"""torch.autograd.Functions over the differentiable batches of the C ABI.

Section 2: DTW is the cost of an optimal warping path, so its gradient is the
gradient of that path's cost, 2(S(i) - T(j)) scattered onto both inputs over
the path cells.  The forward sweeps each pair along its anti-diagonals and,
when a gradient is wanted, records which predecessor gave each cell's minimum
(2 bits per cell); the backward follows that record from the last cell back to
the first and scatters the path's terms.  With recompute=True the forward
keeps no record and the backward sweeps the pairs again.
"""
from __future__ import annotations

import ctypes

import torch


class DTWFunction(torch.autograd.Function):
    """DTW of equal-length pairs S, T [npairs, len] under a window."""

    @staticmethod
    def forward(ctx, S: torch.Tensor, T: torch.Tensor, window: int, recompute: bool = False):
        from . import _dev, _ptr, context
        S32, T32 = _dev(S), _dev(T)
        if S32.shape != T32.shape or S32.dim() != 2:
            raise ValueError("S and T must both be [npairs, len]")
        P, L = S32.shape
        c = context(S32.device.index)
        c.bind_stream()
        want_grad = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        rec = None
        if want_grad and not recompute:
            nbytes = c._lib.eapdtw_dtw_ckpt_bytes(P, L, int(window))
            if nbytes < 0:
                raise ValueError("unsupported sizes for the differentiable batch")
            rec = torch.empty(int(nbytes), device=S32.device, dtype=torch.uint8)
        out = torch.empty(P, device=S32.device, dtype=torch.float32)
        c.check(c._lib.eapdtw_dtw_fwd(c.handle, _ptr(S32), _ptr(T32), P, L, int(window), _ptr(out),
                                      ctypes.c_void_p(rec.data_ptr()) if rec is not None else None))
        ctx.save_for_backward(S32, T32, rec)
        ctx.window = int(window)
        ctx.in_dtypes = (S.dtype, T.dtype)
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        from . import _ptr, context
        S32, T32, rec = ctx.saved_tensors
        P, L = S32.shape
        g = grad_out.to(torch.float32).contiguous()
        c = context(S32.device.index)
        c.bind_stream()
        gS = torch.empty_like(S32)
        gT = torch.empty_like(T32)
        c.check(c._lib.eapdtw_dtw_bwd(c.handle, _ptr(S32), _ptr(T32), P, L, ctx.window,
                                      ctypes.c_void_p(rec.data_ptr()) if rec is not None else None,
                                      _ptr(g), _ptr(gS), _ptr(gT)))
        return gS.to(ctx.in_dtypes[0]), gT.to(ctx.in_dtypes[1]), None, None


class DTWBatchFunction(torch.autograd.Function):
    """DTW of pairs of uneven length and window held in two pools:
    DTWBatchFunction.apply(S_pool, T_pool, pairs, n) with pairs from
    pack_pairs (their regions must not overlap for the backward)."""

    @staticmethod
    def forward(ctx, S_pool: torch.Tensor, T_pool: torch.Tensor, pairs, n: int):
        from . import _dev, _ptr, context
        S32, T32 = _dev(S_pool).reshape(-1), _dev(T_pool).reshape(-1)
        c = context(S32.device.index)
        c.bind_stream()
        rec = None
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            nbytes = c._lib.eapdtw_dtw_batch_record_bytes(pairs, int(n))
            if nbytes < 0:
                raise ValueError("unsupported pairs for the differentiable batch")
            rec = torch.empty(max(int(nbytes), 1), device=S32.device, dtype=torch.uint8)
        out = torch.empty(int(n), device=S32.device, dtype=torch.float32)
        c.check(c._lib.eapdtw_dtw_batch_fwd(
            c.handle, _ptr(S32), S32.numel(), _ptr(T32), T32.numel(), pairs, int(n), _ptr(out),
            ctypes.c_void_p(rec.data_ptr()) if rec is not None else None))
        ctx.save_for_backward(S32, T32, rec)
        ctx.pairs, ctx.n = pairs, int(n)
        ctx.in_dtypes = (S_pool.dtype, T_pool.dtype)
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        from . import _ptr, context
        S32, T32, rec = ctx.saved_tensors
        g = grad_out.to(torch.float32).contiguous()
        c = context(S32.device.index)
        c.bind_stream()
        gS = torch.zeros_like(S32)
        gT = torch.zeros_like(T32)
        c.check(c._lib.eapdtw_dtw_batch_bwd(
            c.handle, _ptr(S32), S32.numel(), _ptr(T32), T32.numel(), ctx.pairs, ctx.n,
            ctypes.c_void_p(rec.data_ptr()), _ptr(g), _ptr(gS), _ptr(gT)))
        return gS.to(ctx.in_dtypes[0]), gT.to(ctx.in_dtypes[1]), None, None
