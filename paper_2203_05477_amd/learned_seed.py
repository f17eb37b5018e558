"""Harvesting training data from the solver and training the seed network on the GPU.

The samples are the faces' features at the start of a step (pond_mlp_features) and the
face frames the plain iteration converged to in that step (pond_mlp_targets), kept for
converged faces that needed at least `hard_iters` iterations plus a random share of the
others. All arithmetic runs in libpond's kernels; torch only holds the device buffers.
"""
from __future__ import annotations

import numpy as np
import torch

from . import pond


def harvest(cfg, fields, steps, precision="fp64", warmup=0, hard_iters=2, easy_share=0.05,
            seed=0, every=1):
    """Run `steps` plain-seed steps, returning device tensors X (n x 64), T (n x 4)."""
    ctx = pond.Context(cfg, fields, precision=precision)
    if warmup:
        ctx.step(warmup)
    nf = ctx.nfaces
    rng = np.random.Generator(np.random.PCG64(seed))
    X = torch.empty((nf, 64), dtype=torch.float32, device="cuda")
    ref = torch.empty((nf, 4), dtype=torch.float32, device="cuda")
    T = torch.empty((nf, 4), dtype=torch.float32, device="cuda")
    xs, ts = [], []
    torch.cuda.synchronize()
    for k in range(steps):
        take = (k % every) == 0
        if take:
            ctx.mlp_features(X.data_ptr(), ref.data_ptr())
        ctx.step(1)
        if not take:
            continue
        ctx.mlp_targets(X.data_ptr(), ref.data_ptr(), T.data_ptr())
        it = ctx.face_iters()
        keep = (it >= hard_iters) | ((it > 0) & (rng.random(nf) < easy_share))
        idx = torch.from_numpy(np.nonzero(keep)[0]).to("cuda")
        xs.append(X.index_select(0, idx))
        ts.append(T.index_select(0, idx))
        torch.cuda.synchronize()  # X, T are rewritten by the library's stream next step
    ctx.close()
    return torch.cat(xs), torch.cat(ts)


def train(datasets, epochs=30, batch=4096, lr=2e-3, seed=0, init=None):
    """Train a seed network on the concatenation of (X, T) datasets (shuffled once)."""
    X = torch.cat([d[0] for d in datasets]).contiguous()
    T = torch.cat([d[1] for d in datasets]).contiguous()
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(X.shape[0], generator=g).to(X.device)
    X = X.index_select(0, perm).contiguous()
    T = T.index_select(0, perm).contiguous()
    net = pond.Mlp(params=init, seed=seed)
    torch.cuda.synchronize()  # the library works on its own stream
    losses = net.train(X.data_ptr(), T.data_ptr(), X.shape[0], epochs=epochs, batch=batch, lr=lr)
    torch.cuda.synchronize()
    return net, losses, X.shape[0]
