"""Pins of the FP64 reference of the seed network (oracle/mlp.py): central finite
differences of the loss, BF16 rounding of known values, and descent."""
import numpy as np

from oracle import mlp as M


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1.0);
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -8 + 2 ** -20, -2.5, 3.0e-3])
    r = M.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6
    assert r[3] == 1.0 + 2 ** -7
    assert r[4] == -2.5
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = M.he_params(1) + 0.01 * rng.standard_normal(M.NPARAM)
    X = np.zeros((7, 64))
    X[:, :40] = rng.standard_normal((7, 40))
    T = rng.standard_normal((7, 4))
    loss, g = M.loss_and_grad(p, X, T)
    idx = rng.choice(M.NPARAM, 60, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros(M.NPARAM)
        e[k] = h
        fd = (M.loss_and_grad(p + e, X, T)[0] - M.loss_and_grad(p - e, X, T)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_gradient_descent_reduces_loss():
    rng = np.random.default_rng(3)
    p = M.he_params(2)
    X = np.zeros((64, 64))
    X[:, :40] = rng.standard_normal((64, 40))
    T = np.zeros((64, 4))
    T[:, 0] = np.tanh(X[:, 0])
    l0, g = M.loss_and_grad(p, X, T)
    l1, _ = M.loss_and_grad(p - 1e-3 * g, X, T)
    assert l1 < l0
