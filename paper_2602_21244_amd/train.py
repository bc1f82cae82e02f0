"""Train the neural collision operator on pairs our own quadrature labels.

Data ("physics harvesting" on synthetic pairs): rows (v_r, xi, z) with g
log-uniform on [100, 20000] m/s and isotropic direction; dsmc_harvest_rows
computes chi(b(z), g) by the quadrature kernel and the target post-collision
relative velocity.  Each step: forward (MFMA), the loss, hand-written
backward, Adam with a cosine learning-rate schedule decaying to 1e-6
(section "Neural Surrogate Training").  Loss "direction" (default): the MSE
on the scattering directions, each pair normalised by its own g^2;
"velocity": the MSE on the post-collision velocities normalised by
sigma_v^2, which weights a pair by (g / sigma_v)^2 and so leaves the
directions of slow pairs (most pairs of a 200 K gas) nearly untrained.

    python -m paper_2602_21244_amd.train --steps 60000 --pool 4194304 \
        --out weights/jager_surrogate_8x128x4.npz
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

from . import api

HERE = os.path.dirname(os.path.abspath(__file__))


def harvest(workloads, n, seed, dev, pot, quad):
    rows = workloads.training_rows(seed=seed, n=n)
    x, g, tgt, chi = api.harvest_rows(torch.as_tensor(rows["vr"], device=dev),
                                      torch.as_tensor(rows["xi"], device=dev),
                                      torch.as_tensor(rows["z"], device=dev),
                                      rows["sigma_v"], workloads.B_MAX, workloads.AR_MASS / 2,
                                      pot, quad)
    return x, g, tgt, chi, rows["sigma_v"]


def direction_error(vr_pred, vr_tgt):
    a = vr_pred.double()
    b = vr_tgt.double()
    c = (a * b).sum(1) / (a.norm(dim=1) * b.norm(dim=1))
    return torch.arccos(torch.clamp(c, -1, 1))


class FlatParams:
    """The network's parameters in one flat FP32 master buffer (with its
    gradient and Adam moments beside it) so that one Adam launch updates all
    of them: the net's bf16 weights become views of one flat bf16 copy that
    Adam rewrites, its fp32 biases views of the master buffer itself."""

    def __init__(self, net, Ws, bs, dev):
        offs, o = [], 0
        for w, b in zip(Ws, bs):
            nw, nb = int(np.prod(w.shape)), int(np.prod(b.shape))
            offs.append((o, nw, o + ((nw + 63) // 64) * 64, nb))
            o = offs[-1][2] + ((nb + 63) // 64) * 64
        self.n = o
        self.master = torch.zeros(o, dtype=torch.float32, device=dev)
        self.grad = torch.zeros_like(self.master)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        for (ow, nw, ob, nb), w, b in zip(offs, Ws, bs):
            self.master[ow:ow + nw] = torch.as_tensor(np.asarray(w, np.float32).ravel(), device=dev)
            self.master[ob:ob + nb] = torch.as_tensor(np.asarray(b, np.float32).ravel(), device=dev)
        self.bf16 = self.master.to(torch.bfloat16)
        self.W, self.b, self.dW, self.db = [], [], [], []
        for (ow, nw, ob, nb), w in zip(offs, Ws):
            shape = tuple(np.asarray(w).shape)
            self.W.append(self.master[ow:ow + nw].view(shape))
            self.b.append(self.master[ob:ob + nb])
            self.dW.append(self.grad[ow:ow + nw].view(shape))
            self.db.append(self.grad[ob:ob + nb])
            net.W[len(self.W) - 1] = self.bf16[ow:ow + nw].view(shape)
            net.b[len(self.b) - 1] = self.master[ob:ob + nb]
        net.refresh()

    def step(self, t, lr):
        api.adam_step(self.master, self.grad, self.m, self.v, t, lr, param_bf16=self.bf16)


def train(steps=4000, batch=65536, pool=1 << 20, lr=2e-3, seed=4, dims=None, out=None,
          log_every=200, dev=None, loss_kind="direction"):
    sys.path.insert(0, os.path.dirname(HERE))
    import workloads as W

    dev = dev or torch.device("cuda:0")
    dims = dims or W.SURROGATE_DIMS
    pot = api.potential_jager(W.JAGER_PLACEHOLDER)
    quad = api.quad_struct(64)
    t0 = time.time()
    x, g, tgt, chi, sigma_v = harvest(W, pool, seed, dev, pot, quad)
    xv, gv, tv, _, _ = harvest(W, 65536, seed + 1000, dev, pot, quad)
    torch.cuda.synchronize()
    print(f"harvested {pool} + 65536 rows in {time.time() - t0:.1f}s", flush=True)
    Ws, bs = W.mlp_init(seed, dims)
    net = api.Net(Ws, bs, act="silu", wdtype="bf16", sigma_v=sigma_v, device=dev)
    params = FlatParams(net, Ws, bs, dev)
    act = api.workspace(api.neural_act_bytes(net, batch), dev)
    bws = api.workspace(api.lib().dsmc_neural_backward_ws(__import__("ctypes").byref(net.struct), batch), dev)
    dvr = torch.empty(batch, 3, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    hist = []
    t0 = time.time()
    for t in range(1, steps + 1):
        idx = torch.randint(0, pool, (batch,), device=dev, generator=gen)
        xb, gb, tb = x[idx].contiguous(), g[idx].contiguous(), tgt[idx].contiguous()
        y, vr = api.neural_forward_rows(net, xb, gb, act_save=act)
        loss.zero_()
        if loss_kind == "direction":
            api.direction_loss(vr, tb, dvr, loss)
        else:
            api.mse_loss(vr, tb, sigma_v, dvr, loss)
        api.neural_backward(net, xb, act, y, gb, dvr, params.dW, params.db, ws=bws)
        lr_t = api.cosine_lr(t, steps, lr)
        params.step(t, lr_t)
        if t % log_every == 0 or t == 1 or t == steps:
            yv, vrv = api.neural_forward_rows(net, xv, gv)
            err = direction_error(vrv, tv)
            rms = float(torch.sqrt((err ** 2).mean()))
            hist.append((t, float(loss.item()), rms))
            print(f"step {t:5d} loss {loss.item():.5f} val dir rms {rms:.4f} rad "
                  f"lr {lr_t:.2e} ({time.time() - t0:.1f}s)", flush=True)
    torch.cuda.synchronize()
    if out:
        os.makedirs(os.path.dirname(out), exist_ok=True)
        arrs = {"n_layers": np.int64(len(net.W)), "sigma_v": np.float64(sigma_v),
                "dims": np.array(dims, np.int64), "history": np.array(hist),
                "steps": np.int64(steps), "lr": np.float64(lr), "pool": np.int64(pool),
                "loss": np.array(loss_kind)}
        for l in range(len(net.W)):
            arrs[f"W{l}"] = params.W[l].double().cpu().numpy()
            arrs[f"b{l}"] = params.b[l].double().cpu().numpy()
        np.savez(out, **arrs)
        print("saved", out, flush=True)
    master = [p for pair in zip(params.W, params.b) for p in pair]
    return net, master, hist


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--steps", type=int, default=4000)
    p.add_argument("--batch", type=int, default=65536)
    p.add_argument("--pool", type=int, default=1 << 20)
    p.add_argument("--lr", type=float, default=2e-3)
    p.add_argument("--seed", type=int, default=4)
    p.add_argument("--loss", default="direction", choices=["direction", "velocity"])
    p.add_argument("--out", default=os.path.join(HERE, "weights", "jager_surrogate_8x128x4.npz"))
    a = p.parse_args()
    train(a.steps, a.batch, a.pool, a.lr, a.seed, out=a.out, loss_kind=a.loss)


if __name__ == "__main__":
    main()
