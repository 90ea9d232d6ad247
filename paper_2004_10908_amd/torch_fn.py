"""torch.autograd.Function over the library's forward and backward passes.

Forward runs sdnn_forward (saving the layer checkpoints every ``ckpt_every``
layers); backward runs sdnn_backward, which recomputes each checkpoint segment
and returns gradients for the input rows, the weight values on the fixed
pattern and the biases.  The index pattern has no gradient.  torch is used only
for device memory and the current stream.
"""
from __future__ import annotations

import torch

from .sdnn import Net


class SparseDNNFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0: torch.Tensor, w: torch.Tensor, bias: torch.Tensor, net: Net):
        if w.data_ptr() != net.w.data_ptr() or bias.data_ptr() != net.bias.data_ptr():
            raise ValueError("w and bias must be the tensors the net was created over")
        y0 = y0.contiguous()
        o = net.forward(y0, ckpt=net.ckpt_every > 0)
        ctx.net = net
        ckpt = o["ckpt"] if o["ckpt"] is not None else torch.empty(1, device=y0.device)
        ctx.save_for_backward(y0, ckpt, o["nz_rows"], o["n_nz"])
        ctx.mark_non_differentiable(o["nz_rows"], o["n_nz"])
        return o["y"], o["nz_rows"], o["n_nz"]

    @staticmethod
    def backward(ctx, dy, _g_nz=None, _g_n=None):
        y0, ckpt, nz_rows, n_nz = ctx.saved_tensors
        net: Net = ctx.net
        dw, db, dy0 = net.backward(y0, ckpt, nz_rows, n_nz, dy.contiguous(), want_dy0=ctx.needs_input_grad[0])
        return dy0, dw, db, None


def sparse_dnn(y0: torch.Tensor, net: Net, w: torch.Tensor = None, bias: torch.Tensor = None):
    """Differentiable forward: returns (y_out, nz_rows, n_nz).

    ``w`` / ``bias`` are the parameter tensors gradients should reach (leaf tensors
    sharing storage with the ones the net was created over); default: the net's own.
    """
    return SparseDNNFunction.apply(y0, net.w if w is None else w, net.bias if bias is None else bias, net)
