"""FP64 reference of the seed network (TEST INFRASTRUCTURE: used only by the tests).

A 2 x 64 hidden-layer ReLU network y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 with the
parameter vector W1 (64x64, out x in), b1, W2 (64x64), b2, W3 (3x64), b3, and the loss
(1/n) sum_s sum_o (y_so - t_so)^2. Written from the definitions of the network and of
reverse-mode differentiation (chain rule, layer by layer). No code is shared with the
GPU library.

`bf16=True` (or a rounding function) evaluates the network the way a BF16-input /
FP32-accumulate pipeline sees it:
weights, inputs and the hidden activations entering the next layer are rounded to BF16
(round to nearest even) and everything else is exact FP64. The gradient is then the exact
gradient of that evaluation with the rounding treated as the identity.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 64, 64, 3
SHAPES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NOUT, NH)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, k = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[k:k + n], dtype=np.float64).reshape(shape)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, X, bf16=False):
    """Outputs (n x 3) and the intermediate values needed by backward."""
    P = unpack(p)
    if callable(bf16):
        rnd = bf16
    else:
        rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, W3 = rnd(P["W1"]), rnd(P["W2"]), rnd(P["W3"])
    x = rnd(X)
    z1 = x @ W1.T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    h1r = rnd(h1)
    z2 = h1r @ W2.T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    h2r = rnd(h2)
    y = h2r @ W3.T + P["b3"]
    return y, dict(x=x, z1=z1, h1=h1r, z2=z2, h2=h2r, W1=W1, W2=W2, W3=W3)


def loss_and_grad(p, X, T, bf16=False):
    """Loss (1/n) sum (y - t)^2 and its gradient w.r.t. the parameter vector."""
    n = X.shape[0]
    y, c = forward(p, X, bf16)
    e = y - np.asarray(T, dtype=np.float64)[:, :NOUT]
    loss = float(np.sum(e * e) / n)
    dy = 2.0 * e / n
    g = {}
    g["W3"] = dy.T @ c["h2"]
    g["b3"] = dy.sum(axis=0)
    dz2 = (dy @ c["W3"]) * (c["z2"] > 0)
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ c["W2"]) * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["x"]
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def he_params(seed=0, nin_used=40):
    """He-normal weights on the used inputs, zero biases (seeded numpy generator)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = {name: np.zeros(shape) for name, shape in SHAPES}
    d["W1"][:, :nin_used] = rng.normal(0.0, np.sqrt(2.0 / nin_used), (NH, nin_used))
    d["W2"] = rng.normal(0.0, np.sqrt(2.0 / NH), (NH, NH))
    d["W3"] = rng.normal(0.0, np.sqrt(2.0 / NH), (NOUT, NH))
    return pack(d)


def loss_and_grad_bf16_pipeline(p, X, T, rnd=bf16_round):
    """Loss and gradient as a BF16-operand / FP32-accumulate training pipeline computes them,
    exact (FP64) except at its rounding points: weights, inputs and the hidden activations
    entering the next layer (as forward(bf16=True)); the output error dY = 2 (y - t)/n
    rounded to BF16 before the layer-3 weight gradient (the back-propagation dY W3 and the
    bias gradient use it unrounded); the back-propagated dZ2 and dZ1 rounded to BF16 before
    every product and sum that uses them. Returns the loss, the gradient and the
    intermediates (for error bounds). `rnd` is the rounding applied at those points (the
    identity turns the pipeline into the exact network and gradient)."""
    n = X.shape[0]
    y, c = forward(p, X, bf16=rnd)
    e = y - np.asarray(T, dtype=np.float64)[:, :NOUT]
    loss = float(np.sum(e * e) / n)
    dy = 2.0 * e / n
    dyb = rnd(dy)
    g = {}
    g["W3"] = dyb.T @ c["h2"]
    g["b3"] = dy.sum(axis=0)
    d2 = (dy @ c["W3"]) * (c["z2"] > 0)
    D2 = rnd(d2)
    g["W2"] = D2.T @ c["h1"]
    g["b2"] = D2.sum(axis=0)
    d1 = (D2 @ c["W2"]) * (c["z1"] > 0)
    D1 = rnd(d1)
    g["W1"] = D1.T @ c["x"]
    g["b1"] = D1.sum(axis=0)
    c.update(y=y, e=e, dy=dy, dyb=dyb, d2=d2, D2=D2, d1=d1, D1=D1)
    return loss, pack(g), c
