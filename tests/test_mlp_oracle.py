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


def test_bf16_pipeline_reference():
    """The BF16-pipeline gradient: with the identity at its rounding points it is the exact
    network gradient (pinned above by finite differences); with BF16 rounding it stays within
    a few BF16 units (2^-8 relative) of the exact gradient of the BF16 forward evaluation, and
    each of its rounding points matters (rounding dZ1 alone changes the layer-1 gradient)."""
    rng = np.random.default_rng(4)
    p = M.he_params(3) + 0.01 * rng.standard_normal(M.NPARAM)
    X = np.zeros((33, 64))
    X[:, :40] = rng.standard_normal((33, 40))
    T = rng.standard_normal((33, 4))
    ident = lambda a: np.asarray(a, dtype=np.float64)  # noqa: E731
    l0, g0, _ = M.loss_and_grad_bf16_pipeline(p, X, T, rnd=ident)
    l1, g1 = M.loss_and_grad(p, X, T)
    assert l0 == l1 and np.array_equal(g0, g1)
    lb, gb, c = M.loss_and_grad_bf16_pipeline(p, X, T)
    lf, gf = M.loss_and_grad(p, X, T, bf16=True)
    assert lb == lf
    assert 0 < np.linalg.norm(gb - gf) <= 4 * 2 ** -8 * np.linalg.norm(gf)
    # the layer-1 weight gradient is D1^T x with D1 = bf16(dZ1)
    gW1 = M.unpack(gb)["W1"]
    assert np.allclose(gW1, c["D1"].T @ c["x"], rtol=1e-14, atol=0)
    assert not np.allclose(gW1, c["d1"].T @ c["x"], rtol=1e-6, atol=0)
