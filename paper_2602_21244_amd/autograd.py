"""torch.autograd.Function wrappers around the hand-written forward/backward
kernels of the surrogate (rows form: x -> y = f_theta(x) -> v_r' = g y/|y|)
and of the cell-wise moment matching (v -> u_pre + alpha (v - u_post))."""
from __future__ import annotations

import torch

from . import api


class SurrogateFn(torch.autograd.Function):
    """y_raw, vr' = f(x, g; theta).  The parameters enter through `net` (its
    device weights); the returned gradients are for the tensors in `params`
    (one W and one b per layer, in order), which must be the FP32 (BF16 net) or
    FP64 (FP64 net) master copies of net's weights.  Only vr' is
    differentiable: y_raw is returned for inspection (the backward kernel
    takes dL/dvr' and forms the projection adjoint itself)."""

    @staticmethod
    def forward(ctx, x, g, net, *params):
        act = api.workspace(api.neural_act_bytes(net, x.shape[0]), x.device)
        y, vr = api.neural_forward_rows(net, x, g, act_save=act)
        ctx.net = net
        ctx.save_for_backward(x, g, y)
        ctx.act = act
        ctx.mark_non_differentiable(y)
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


class MomentMatchFn(torch.autograd.Function):
    """Centred cell-wise moment matching (eq. cell_energy_clamp, centred
    reading) of FP64 SoA velocities v[3][n] in cell-sorted order: each cell
    with N >= 2 and S_post > 0 becomes u_pre + alpha (v - u_post), alpha =
    sqrt(S_pre / S_post), with the pre-collision moments `mom_pre` (from
    dsmc_moment_match CAPTURE) held fixed.  The backward is the adjoint
    kernel dsmc_moment_match_backward."""

    @staticmethod
    def forward(ctx, v_post, cell_start, mom_pre):
        out = v_post.detach().clone().contiguous()
        api.moment_match(cell_start, out, mom_pre, api.L.MM_APPLY)
        ctx.save_for_backward(v_post.detach().contiguous(), cell_start, mom_pre)
        return out

    @staticmethod
    def backward(ctx, G):
        v_post, cs, mom = ctx.saved_tensors
        return api.moment_match_backward(cs, mom, v_post, G.contiguous()), None, None


def moment_match(v_post, cell_start, mom_pre):
    return MomentMatchFn.apply(v_post, cell_start, mom_pre)
