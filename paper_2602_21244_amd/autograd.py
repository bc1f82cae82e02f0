"""torch.autograd.Function around the hand-written forward/backward kernels of
the surrogate (rows form: x -> y = f_theta(x) -> v_r' = g y/|y|)."""
from __future__ import annotations

import torch

from . import api


class SurrogateFn(torch.autograd.Function):
    """y_raw, vr' = f(x, g; theta).  The parameters enter through `net` (its
    device weights); the returned gradients are for the tensors in `params`
    (one W and one b per layer, in order), which must be the FP32 (BF16 net) or
    FP64 (FP64 net) master copies of net's weights."""

    @staticmethod
    def forward(ctx, x, g, net, *params):
        act = api.workspace(api.neural_act_bytes(net, x.shape[0]), x.device)
        y, vr = api.neural_forward_rows(net, x, g, act_save=act)
        ctx.net = net
        ctx.save_for_backward(x, g, y)
        ctx.act = act
        ctx.param_shapes = [p.shape for p in params]
        return vr, y

    @staticmethod
    def backward(ctx, dvr, dy_unused):
        x, g, y = ctx.saved_tensors
        net = ctx.net
        gt = torch.float64 if net.wdtype == "f64" else torch.float32
        dW = [torch.zeros(tuple(w.shape), dtype=gt, device=x.device) for w in net.W]
        db = [torch.zeros(tuple(b.shape), dtype=gt, device=x.device) for b in net.b]
        dx = torch.zeros_like(x)
        api.neural_backward(net, x, ctx.act, y, g, dvr.contiguous().to(gt), dW, db, dx=dx)
        grads = []
        for l in range(len(net.W)):
            grads.append(dW[l])
            grads.append(db[l])
        return (dx, None, None, *grads)


def surrogate(net, x, g, params):
    return SurrogateFn.apply(x, g, net, *params)
