"""torch.autograd wrappers of the deformation path (argument marshalling only).

``DeformField`` describes one scene's field (grid, decoder shape, precision form);
``Hash4DDeform.apply(xyzt, table, params, field, scaler)`` returns the decoder output
delta = [dx | drot | dscale] (DASH Section 4.2) and routes its backward through the
library's decoder backward and table scatter (and, when the positions require a
gradient, the encoder's input gradient); ``SmoothnessReg.apply(xyzt, eps,
table, field, lam)`` returns the Eq. 11 regulariser, whose table gradient the
library computes in the same pass as the loss.

``table`` [E, F] and ``params`` (flat) are the FP32 masters (FP64 for the FP64
check form).  In the BF16 form the BF16 copies are made by the library's rounding
kernel on every call, and gradients come back in FP32, unscaled.
"""
from __future__ import annotations

import torch

from . import _lib


class DeformField:
    def __init__(self, grid: _lib.Grid, mlp: _lib.Mlp, dtype: int = _lib.F32):
        self.grid, self.mlp, self.dtype = grid, mlp, dtype

    @property
    def torch_dtype(self):
        return torch.float64 if self.dtype == _lib.F64 else torch.float32

    def lowered(self, t: torch.Tensor) -> torch.Tensor:
        """The tensor the kernels read: a fresh BF16 copy in the BF16 form."""
        t = t.detach().contiguous()
        if self.dtype != _lib.BF16:
            return t
        lo = torch.empty(t.numel(), dtype=torch.int16, device=t.device)
        _lib.h4d_cast_bf16(t, lo, t.numel())
        return lo


class Hash4DDeform(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyzt, table, params, field: DeformField, scaler=None):
        g, m = field.grid, field.mlp
        n = xyzt.shape[0]
        xyzt = xyzt.detach().contiguous()
        t_used, p_used = field.lowered(table), field.lowered(params)
        feat = torch.empty((g.L, n, g.F), dtype=field.torch_dtype, device=xyzt.device)
        delta = torch.empty((n, m.out), dtype=field.torch_dtype, device=xyzt.device)
        _lib.hash4d_deform_forward(g, m, field.dtype, t_used, p_used, xyzt, n, feat, delta)
        ctx.save_for_backward(xyzt, feat, p_used, t_used)
        ctx.field, ctx.scaler = field, scaler
        ctx.table_shape, ctx.n_params = tuple(table.shape), params.numel()
        return delta

    @staticmethod
    def backward(ctx, d_delta):
        xyzt, feat, p_used, t_used = ctx.saved_tensors
        field, scaler = ctx.field, ctx.scaler
        g, m = field.grid, field.mlp
        n = xyzt.shape[0]
        dev = xyzt.device
        S = scaler.scale if scaler is not None else 1.0
        d_table = torch.zeros(ctx.table_shape, dtype=field.torch_dtype, device=dev)
        d_params = torch.zeros(ctx.n_params, dtype=field.torch_dtype, device=dev)
        d_delta = d_delta.to(field.torch_dtype).contiguous()
        if not ctx.needs_input_grad[0]:
            ws_bytes = _lib.hash4d_deform_workspace_bytes(g, m, field.dtype, n)
            ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
            _lib.hash4d_deform_backward(g, m, field.dtype, p_used, xyzt, n, feat, d_delta, S, 1.0 / S, d_table,
                                        d_params, ws, ws_bytes)
            d_xyzt = None
        else:
            # the positions need their gradient too (the derivative of Eq. 9 with
            # respect to x): decoder backward, then the table scatter and the input
            # gradient from the same (unscaled) feature gradient
            LM = _lib.LEVEL_MAJOR
            d_feat = torch.empty((g.L, n, g.F), dtype=field.torch_dtype, device=dev)
            wb = _lib.deform_mlp_workspace_bytes(m, field.dtype, n)
            ws = torch.empty(max(wb, 1), dtype=torch.uint8, device=dev)
            _lib.deform_mlp_backward(m, field.dtype, p_used, feat, n, d_delta, S, 1.0 / S, d_feat, d_params, ws, wb,
                                     LM, g.F)
            grad_dt = _lib.F64 if field.dtype == _lib.F64 else _lib.F32
            wb = _lib.hash4d_encode_backward_workspace_bytes(g, n)
            ws = torch.empty(max(wb, 1), dtype=torch.uint8, device=dev)
            _lib.hash4d_encode_backward(g, grad_dt, xyzt, n, d_feat, 1.0, d_table, ws, wb, LM)
            d_xyzt = torch.zeros((n, 4), dtype=field.torch_dtype, device=dev)
            wb = _lib.hash4d_encode_backward_input_workspace_bytes(g, field.dtype, n)
            ws = torch.empty(max(wb, 1), dtype=torch.uint8, device=dev) if wb else None
            _lib.hash4d_encode_backward_input(g, field.dtype, t_used, xyzt, n, d_feat, 1.0, d_xyzt, LM, ws, wb)
            d_xyzt = d_xyzt.to(xyzt.dtype)
        if scaler is not None:
            scaler.observe(d_table, d_params)
        return d_xyzt, d_table, d_params, None, None


class SmoothnessReg(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyzt, eps, table, field: DeformField, lam: float = 1.0):
        g = field.grid
        n = xyzt.shape[0]
        loss = torch.zeros(1, dtype=field.torch_dtype, device=xyzt.device)
        d_table, ws, wb = None, None, 0
        if table.requires_grad:
            d_table = torch.zeros(tuple(table.shape), dtype=field.torch_dtype, device=xyzt.device)
            wb = _lib.smoothness_workspace_bytes(g, field.dtype, n)
            ws = torch.empty(max(wb, 1), dtype=torch.uint8, device=xyzt.device)
        _lib.smoothness_reg(g, field.dtype, field.lowered(table), xyzt.detach().contiguous(),
                            eps.detach().contiguous(), n, lam, loss, d_table, ws, wb)
        ctx.save_for_backward(d_table if d_table is not None else loss)
        ctx.has_grad = d_table is not None
        return loss[0]

    @staticmethod
    def backward(ctx, g_loss):
        (d_table,) = ctx.saved_tensors
        return None, None, (g_loss * d_table if ctx.has_grad else None), None, None
