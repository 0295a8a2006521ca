"""Training and evaluation driver of the learned work estimator.

The network (8 -> 64 -> 64 -> 1, ReLU, float16 weights, float32 arithmetic)
predicts y = log2(1 + n_pc + n_pp) of a group from the features that
mibh_group_features computes.  Training pairs come from the walk itself (its
exact per-group interaction counts); forward, backward and Adam run in the
library's HIP kernels (mibh_mlp_*).  This module only allocates buffers, draws
mini-batch indices and loops.
"""
from __future__ import annotations

import math

import numpy as np

from . import mibh

VERSION = 1


def collect(ctx, theta: float):
    """(features [G,8], targets [G]) of the context's current tree after compute_forces(theta)."""
    import torch
    feat = ctx.group_features(theta).clone()
    counts = ctx.export("counts").view(torch.int32).reshape(-1, 2).to(torch.float64)
    target = torch.log2(1.0 + counts[:, 0] + counts[:, 1]).to(torch.float32)
    return feat, target


def init_weights(device, seed: int = 0):
    """He-initialised float32 master weights (layout of MIBH_MLP_PARAMS) and a float16 copy."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    parts = [torch.randn(64, 8, generator=g) * math.sqrt(2.0 / 8), torch.zeros(64),
             torch.randn(64, 64, generator=g) * math.sqrt(2.0 / 64), torch.zeros(64),
             torch.randn(64, generator=g) * math.sqrt(1.0 / 64), torch.full((1,), 10.0)]
    w32 = torch.cat([p.reshape(-1) for p in parts]).to(torch.float32).to(device)
    assert w32.numel() == mibh.MLP_PARAMS
    return w32, w32.to(torch.float16)


def train(x, t, steps: int = 2000, batch: int = 1024, lr: float = 3e-3, seed: int = 0, w32=None):
    """Adam on the mean squared error of log2 interaction counts.  Returns (w32, w16, losses)."""
    import torch
    dev = x.device
    if w32 is None:
        w32, w16 = init_weights(dev, seed)
    else:
        w16 = w32.to(torch.float16)
    m = torch.zeros_like(w32)
    v = torch.zeros_like(w32)
    grad = torch.empty_like(w32)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    scratch = torch.empty(int(mibh.lib().mibh_mlp_scratch_bytes(batch)), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev).manual_seed(seed)
    losses = []
    n = int(x.shape[0])
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (batch,), generator=gen, device=dev, dtype=torch.int32)
        mibh.mlp_gradient(w16, x, t, idx, grad, loss, scratch)
        step_lr = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps))  # cosine decay
        mibh.mlp_adam(w32, w16, grad, m, v, step, step_lr)
        if step % 100 == 0 or step == 1:
            losses.append((step, float(loss.item())))
    return w32, w16, losses


def evaluate(w16, x, t, margin: float = 1.25):
    """Prediction quality, scored against the exact counts: MAPE of the
    interaction count, RMS error of log2, and the misprediction rate (exact
    count above margin x predicted count)."""
    import torch
    y = mibh.mlp_forward(w16, x)
    pred = torch.exp2(y.double()) - 1.0
    true = torch.exp2(t.double()) - 1.0
    mape = float(torch.mean(torch.abs(pred - true) / torch.clamp(true, min=1.0)))
    rms = float(torch.sqrt(torch.mean((y.double() - t.double()) ** 2)))
    miss = float(torch.mean((true > margin * pred).double()))
    return {"mape": mape, "rms_log2": rms, "mispredict_rate": miss, "margin": margin}


def save(path: str, w32, meta: dict | None = None):
    np.savez(path, w32=w32.detach().cpu().numpy(), version=VERSION,
             features="log2(n)/6,log2(ext/L)/24,log2(dist/L)/24,log2(rel_density)/32,theta,level/20,"
                      "log2(N)/24,log2(theta)", **(meta or {}))


def load(path: str, device):
    import torch
    d = np.load(path, allow_pickle=False)
    if int(d["version"]) != VERSION:
        raise ValueError("estimator weights of another version")
    w32 = torch.from_numpy(d["w32"]).to(device)
    return w32, w32.to(torch.float16)
