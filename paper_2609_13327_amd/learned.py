"""Host-side driver of the learned warm start: it sequences library calls only
(every product, loss, gradient and Adam update runs in libpcsqrt's kernels).

make_pairs: training pairs (b = Z^T x, y = Z^+ x) from a plan's direct solve,
    with x drawn on the device from a seeded generator; stored as the
    network's normalized inputs b / ||b|| and targets y / ||b||.
train: Adam on the relative mean-squared error over minibatches of the
    training rows, with the last `n_val` rows held out: the validation loss
    is evaluated every `eval_every` steps, the learning rate halves when it
    has not improved for `patience` evaluations, and the parameters with the
    lowest validation loss are kept (early stopping).  A network whose output
    layer starts at zero predicts y = 0 (loss 1, the zero start), so the kept
    network is never worse than the zero start on the validation rows.
"""
from __future__ import annotations

import numpy as np

from . import (Mlp, pc_mlp_get_params, pc_mlp_gradients, pc_mlp_set_params, pc_mlp_train_step,
               pc_mlp_training_pairs, pc_sqrt_transpose_apply)


def make_pairs(plan, n: int, KM: int, count: int, seed: int, chunk: int = 1024):
    import torch
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    Xin = torch.empty((count, KM), dtype=torch.float32, device=dev)
    Tin = torch.empty_like(Xin)
    Bc = torch.empty((chunk, KM), dtype=torch.float64, device=dev).t()
    Yc = torch.empty((chunk, KM), dtype=torch.float64, device=dev).t()
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk)
        Xc = torch.randn((c1 - c0, n), generator=g, dtype=torch.float64, device=dev).t()
        pc_sqrt_transpose_apply(plan.handle, 0, Xc, Bc[:, :c1 - c0])
        plan.apply([Xc], [Yc[:, :c1 - c0]])
        pc_mlp_training_pairs(Bc[:, :c1 - c0], Yc[:, :c1 - c0], Xin[c0:c1], Tin[c0:c1])
    return Xin, Tin


def new_network(d: int, h: int, max_batch: int, seed: int, operand: int):
    """Network with W1 ~ N(0, 1/d) (seeded) and a zero output layer."""
    import torch
    import workloads as wl
    W1, b1, _, _ = wl.mlp_init(d, h, seed)
    net = Mlp(d, h, max_batch, operand)
    f32 = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda:0")
    pc_mlp_set_params(net.handle, f32(W1), f32(b1), torch.zeros((d, h), dtype=torch.float32, device="cuda:0"),
                      torch.zeros(d, dtype=torch.float32, device="cuda:0"))
    return net


def validation_loss(net, Xv, Tv, batch: int) -> float:
    import torch
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    tot, cnt = 0.0, 0
    for r0 in range(0, Xv.shape[0], batch):
        r1 = min(Xv.shape[0], r0 + batch)
        pc_mlp_gradients(net.handle, Xv[r0:r1], Tv[r0:r1], loss, None, None, None, None)
        tot += float(loss.item()) * (r1 - r0)
        cnt += r1 - r0
    return tot / max(cnt, 1)


def train(net, Xin, Tin, n_val: int, batch: int = 256, lr: float = 1e-3, max_steps: int = 2000,
          eval_every: int = 50, patience: int = 4, log=None):
    import torch
    d, h = net.d, net.h
    N = Xin.shape[0] - n_val
    Xt, Tt, Xv, Tv = Xin[:N], Tin[:N], Xin[N:], Tin[N:]
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    best = [torch.empty((h, d), dtype=torch.float32, device="cuda:0"),
            torch.empty(h, dtype=torch.float32, device="cuda:0"),
            torch.empty((d, h), dtype=torch.float32, device="cuda:0"),
            torch.empty(d, dtype=torch.float32, device="cuda:0")]
    pc_mlp_get_params(net.handle, *best)
    best_val = validation_loss(net, Xv, Tv, batch)
    history = [(0, None, best_val)]
    stale = 0
    order = torch.randperm(N, generator=torch.Generator().manual_seed(5002)).to("cuda:0")
    pos = 0
    for step in range(1, max_steps + 1):
        if pos + batch > N:
            order = order[torch.randperm(N, generator=torch.Generator().manual_seed(5002 + step)).to("cuda:0")]
            pos = 0
        idx = order[pos:pos + batch]
        pos += batch
        pc_mlp_train_step(net.handle, Xt[idx].contiguous(), Tt[idx].contiguous(), lr, loss)
        if step % eval_every == 0 or step == max_steps:
            v = validation_loss(net, Xv, Tv, batch)
            history.append((step, round(float(loss.item()), 5), round(v, 5)))
            if log:
                log(f"  step {step}: training loss {float(loss.item()):.4f}, validation loss {v:.4f}, lr {lr:.2e}")
            if v < best_val:
                best_val, stale = v, 0
                pc_mlp_get_params(net.handle, *best)
            else:
                stale += 1
                if stale >= patience:
                    lr *= 0.5
                    stale = 0
                    if lr < 1e-6:
                        break
    pc_mlp_set_params(net.handle, *best)
    return best_val, history
