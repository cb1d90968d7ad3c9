"""Training driver of the learned scatter surrogate (orchestration only).

For each attenuation map the caller supplies, a learned-scatter context
(scatter_model 2; samples need only its line integrals and scatter-point
factors, so it never builds a path table or band) is made and
lmosem_surrogate_samples turns the
caller's (pixel, angle, u_bin, energy) draws into network inputs and exact
targets;
the samples of all maps are shuffled with the caller's permutation and the
network is trained by the library's own forward, backward and Adam kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lmosem as L


def make_samples(geom: dict, maps, draws, device) -> tuple:
    """Inputs and targets for every (map, draws) pair, concatenated on the GPU."""
    Xs, ts = [], []
    for mu, s in zip(maps, draws):
        ctx = L.Context(dict(geom, scatter_model=2), torch.as_tensor(mu, device=device))
        try:
            X, t = L.lmosem_surrogate_samples(ctx.handle, *[torch.as_tensor(s[k], device=device)
                                                            for k in ("pixel", "angle", "u_bin", "energy")])
        finally:
            ctx.close()
        Xs.append(X)
        ts.append(t)
    return torch.cat(Xs), torch.cat(ts)


def train(init_params: dict, X: torch.Tensor, t: torch.Tensor, perm: np.ndarray, batch=4096, epochs=40,
          lr=2e-3, lr_decay=0.93):
    """New network from init_params, trained on the samples in the order
    given by perm; returns (network handle, per-epoch mean loss)."""
    idx = torch.as_tensor(perm, device=X.device)
    Xp, tp = X[idx].contiguous(), t[idx].contiguous()
    net = L.lmosem_net_create(init_params)
    loss = L.lmosem_net_train(net, Xp, tp, batch=batch, epochs=epochs, lr=lr, lr_decay=lr_decay)
    return net, loss


def mse(net, X: torch.Tensor, t: torch.Tensor) -> float:
    """Mean-squared error of the network on held-out samples."""
    y = torch.empty_like(t)
    L.lmosem_net_forward(net, X.contiguous(), y)
    return float(((y - t) ** 2).mean())
