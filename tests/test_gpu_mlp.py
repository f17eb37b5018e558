"""GPU tests of the seed network: BF16-MFMA forward and backward kernels against the FP64
reference (oracle/mlp.py) evaluated with the same BF16 roundings, training, features, and
the learned seed inside the step.

Tolerances: the kernels round weights, inputs and hidden activations (and, in training,
the output error and dZ2, dZ1) to BF16 and accumulate in FP32; the references apply the same
roundings in FP64. Outputs and gradients are compared element by element, against bounds
propagated from the BF16 ulps of the rounded operands and the FP32 accumulation (a factor
2 of margin on top).
"""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, 64), dtype=np.float32)
    X[:, :40] = rng.standard_normal((n, 40)).astype(np.float32)
    T = np.zeros((n, 4), dtype=np.float32)
    T[:, 0] = np.tanh(X[:, 0] - 0.5 * X[:, 5])
    T[:, 1] = 0.3 * X[:, 2] * X[:, 3]
    T[:, 2] = np.log1p(X[:, 7] ** 2)
    return X, T


U32 = 2.0 ** -24  # FP32 unit roundoff


def _gamma(k):
    return k * U32 / (1.0 - k * U32)


def _ulp_bf16(v):
    """Spacing of BF16 numbers at |v| (8 significant bits): 2^(e - 7), 0 for v = 0."""
    a = np.abs(v)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, 2.0 ** (e - 7), 0.0)


def _rounded_diff(v, E):
    """Bound on |bf16(a) - bf16(v)| over all a with |a - v| <= E: 0 when no BF16 rounding
    midpoint lies within E of v (both round to the same BF16 number), else E plus two BF16
    steps (the rounded values are at most one step apart beyond E; two covers a binade
    edge)."""
    a = np.abs(v)
    u = _ulp_bf16(a)
    q = np.where(u > 0, a / np.where(u > 0, u, 1.0), 0.0)
    dist = np.abs(q - np.floor(q) - 0.5) * u
    # crossing a power of two changes the spacing: treat it as a possible flip too
    p2 = 2.0 ** np.floor(np.log2(np.where(a > 0, a, 1.0)))
    near = (dist <= E) | (a - E <= p2) | (a == 0)
    return np.where(near, E + 2.0 * _ulp_bf16(a + E), 0.0)


def _relu_rounded_diff(z, E):
    """The same for bf16(max(z, 0)): near z = 0 one side may be 0 and the other positive."""
    return np.where(np.abs(z) <= E, np.abs(z) + E + _ulp_bf16(np.abs(z) + E),
                    np.where(z > 0, _rounded_diff(z, E), 0.0))


def _forward_bounds(c, P):
    """Element-wise bounds on |kernel - reference| of the hidden activations and outputs.
    Each layer's pre-activation is a dot product of BF16 operands (exact products) summed
    in FP32 (at most 65 roundings with the bias: gamma(65) times the sum of magnitudes),
    plus what the inputs' own differences carry through |W|; an activation rounded to BF16
    then matches the reference's exactly unless a rounding midpoint (or zero, for the
    ReLU) lies within that bound."""
    W1, W2, W3 = np.abs(c["W1"]), np.abs(c["W2"]), np.abs(c["W3"])
    E1 = _gamma(65) * (np.abs(c["x"]) @ W1.T + np.abs(P["b1"]))
    D1 = _relu_rounded_diff(c["z1"], E1)
    E2 = D1 @ W2.T + _gamma(65) * ((np.abs(c["h1"]) + D1) @ W2.T + np.abs(P["b2"]))
    D2 = _relu_rounded_diff(c["z2"], E2)
    Ey = D2 @ W3.T + _gamma(65) * ((np.abs(c["h2"]) + D2) @ W3.T + np.abs(P["b3"]))
    return E1, D1, E2, D2, Ey


def test_forward_matches_reference():
    """Outputs element by element within the bound propagated from the BF16 ulps of the
    activations and the FP32 accumulation."""
    import torch

    from oracle import mlp as M
    from paper_2203_05477_amd import pond

    p = M.he_params(5).astype(np.float32)
    p[M.NPARAM - 3:] = [0.1, -0.2, 0.3]
    net = pond.Mlp(params=p)
    P = M.unpack(p)
    for n in (1, 16, 37, 1000):
        X, _ = _data(n, n)
        Xd = torch.from_numpy(X).cuda()
        Yd = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        net.forward(Xd.data_ptr(), n, Yd.data_ptr())
        y = Yd.cpu().numpy()[:, :3].astype(np.float64)
        ref, c = M.forward(p, X, bf16=True)
        bound = _forward_bounds(c, P)[-1]
        err = np.abs(y - ref)
        print("forward", n, "max err/bound", (err / bound).max(), "median bound/|y|",
              np.median(bound / np.maximum(np.abs(ref), 1e-30)), flush=True)
        assert np.all(err <= 2.0 * bound)
        assert np.all(Yd.cpu().numpy()[:, 3] == 0.0)


def test_gradient_matches_reference():
    """Loss and every gradient component against the FP64 reference of the same BF16
    pipeline (oracle.mlp.loss_and_grad_bf16_pipeline), within bounds propagated layer by
    layer from the forward bounds: the output error and dZ2, dZ1 are rounded to BF16 (one
    ulp where the two sides round differently), a ReLU mask may flip where a pre-activation
    lies within its bound of zero, and the sums over the n samples (MFMA chunks, per-wave
    partials, the fixed-order reduction) carry at most gamma(n + 64) of the sum of the terms'
    magnitudes."""
    import torch

    from oracle import mlp as M
    from paper_2203_05477_amd import pond

    p = M.he_params(7).astype(np.float32)
    net = pond.Mlp(params=p)
    P = M.unpack(p)
    for n in (32, 50, 4096):
        X, T = _data(n, 100 + n)
        Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
        torch.cuda.synchronize()
        g, loss = net.grad(Xd.data_ptr(), Td.data_ptr(), n)
        lref, gref, c = M.loss_and_grad_bf16_pipeline(p, X, T)
        E1, D1, E2, D2, Ey = _forward_bounds(c, P)
        gs = _gamma(n + 64)
        W2, W3 = np.abs(c["W2"]), np.abs(c["W3"])
        e, dy, dyb = c["e"], c["dy"], c["dyb"]
        Edy = 2.0 * Ey / n + 4 * U32 * np.abs(dy)
        Ddyb = _rounded_diff(dy, Edy)
        b = {}
        b["W3"] = (Ddyb.T @ (np.abs(c["h2"]) + D2) + np.abs(dyb).T @ D2
                   + gs * np.abs(dyb).T @ np.abs(c["h2"]))
        b["b3"] = Edy.sum(axis=0) + gs * np.abs(dy).sum(axis=0)
        raw2 = np.abs(dy) @ W3
        Ed2 = np.where(np.abs(c["z2"]) <= E2, raw2 + Edy @ W3, (Edy @ W3 + _gamma(4) * raw2))
        DD2 = _rounded_diff(c["d2"], Ed2)
        D2a = np.abs(c["D2"])
        b["W2"] = DD2.T @ (np.abs(c["h1"]) + D1) + D2a.T @ D1 + gs * D2a.T @ np.abs(c["h1"])
        b["b2"] = DD2.sum(axis=0) + gs * D2a.sum(axis=0)
        raw1 = D2a @ W2
        Ed1 = np.where(np.abs(c["z1"]) <= E1, raw1 + DD2 @ W2,
                       DD2 @ W2 + _gamma(65) * (raw1 + DD2 @ W2))
        DD1 = _rounded_diff(c["d1"], Ed1)
        D1a = np.abs(c["D1"])
        b["W1"] = DD1.T @ np.abs(c["x"]) + gs * D1a.T @ np.abs(c["x"])
        b["b1"] = DD1.sum(axis=0) + gs * D1a.sum(axis=0)
        bound = M.pack(b)
        err = np.abs(g.astype(np.float64) - gref)
        lb = (2.0 * np.abs(e) * Ey + Ey * Ey).sum() / n + _gamma(n + 64) * (e * e).sum() / n
        print("grad", n, "max err/bound", (err / np.maximum(bound, 1e-300)).max(),
              "median bound/|g|", np.median(bound[gref != 0] / np.abs(gref[gref != 0])),
              "loss", loss, lref, flush=True)
        assert np.all(err <= 2.0 * bound)
        assert abs(loss - lref) <= 2.0 * lb


def test_training_reduces_loss():
    import torch

    from paper_2203_05477_amd import pond

    X, T = _data(20000, 9)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    torch.cuda.synchronize()
    net = pond.Mlp(seed=3)
    _, l0 = net.grad(Xd.data_ptr(), Td.data_ptr(), X.shape[0])
    losses = net.train(Xd.data_ptr(), Td.data_ptr(), X.shape[0], epochs=15, batch=1024, lr=3e-3)
    _, l1 = net.grad(Xd.data_ptr(), Td.data_ptr(), X.shape[0])
    print("train", l0, losses[-1], l1, flush=True)
    assert l1 < 0.3 * l0
    assert losses[-1] < losses[0]


def test_features_of_uniform_flow_are_zero():
    import torch

    from paper_2203_05477_amd import pond

    cfg, f = W.uniform(2, 20, 12, tol=1e-12)
    g = pond.Context(cfg, f, precision="fp64")
    g.step(1)
    nf = g.nfaces
    X = torch.zeros((nf, 64), device="cuda")
    ref = torch.zeros((nf, 4), device="cuda")
    torch.cuda.synchronize()
    g.mlp_features(X.data_ptr(), ref.data_ptr())
    x = X.cpu().numpy()
    assert np.abs(x[:, :39]).max() < 1e-6     # every cell equals the centre; seed = cell frame
    assert np.all(x[:, 39] == 1.0) and np.all(x[:, 40:] == 0.0)
    r = ref.cpu().numpy()
    nfx = 21 * 12
    assert np.allclose(r[:nfx, 0], 0.3) and np.allclose(r[nfx:, 0], -0.2)   # normal velocity
    assert np.allclose(r[:, 3], 0.7)


def test_learned_seed_in_the_step(tmp_path):
    """A seed network trained on face frames the solver itself produces (a y-uniform strip
    of the 400-cell shock tube and a 192 x 48 double Mach run), then one step from the same
    state three ways: the plain seed (previous face frames), the learned seed, and every
    face seeded with the frame the plain run converged to (the best any seed can do).

    Measured on the faces the network seeds (two or more iterations in the previous step)
    that converged in the plain run: the converged-frame seed needs exactly one iteration
    there (one corrector confirms a fixed point), so no seed can save more than the plain
    run's iterations minus one; the learned seed's iterations are reported against that
    bound. The seed does not change what the iteration converges to: faces converged in
    both runs end within a few tolerances of each other."""
    import torch

    from paper_2203_05477_amd import learned_seed as LS
    from paper_2203_05477_amd import pond

    tol = 1e-10
    cfg, f = W.double_mach(192, 48, tol=tol)
    c1, f1 = W.shock_tube(400, tol=tol)
    cs, fs = W.strip_2d(c1, f1, ny=4)
    data = [LS.harvest(cfg, f, steps=60, precision="fp64", hard_iters=2),
            LS.harvest(cs, fs, steps=200, precision="fp64", hard_iters=2)]
    net, losses, n = LS.train(data, epochs=20, batch=1024, lr=2e-3)
    print("samples", n, "loss", losses[0], losses[-1], flush=True)
    assert losses[-1] < losses[0]
    base = pond.Context(cfg, f, precision="fp64")
    base.step(30)
    seeded = np.abs(base.face_iters()) >= 2
    path = tmp_path / "s.ckpt"
    base.save(path)
    base.close()

    def one_step(seed, frames=None):
        ctx = pond.Context(cfg, f, precision="fp64", seed=seed)
        if seed == "mlp":
            ctx.load_mlp(net, hard_iters=2)
        ctx.load_state(path)
        if frames is not None:
            ctx.set_face_frames(frames)
        ctx.step(1)
        out = ctx.face_iters(), ctx.face_frames()
        ctx.close()
        return out

    it_p, fr_p = one_step("prev")
    it_l, fr_l = one_step("mlp")
    it_c, _ = one_step("prev", fr_p)
    sel = seeded & (it_p > 0)
    assert sel.sum() >= 20
    m_p, m_l, m_c = it_p[sel].mean(), np.abs(it_l[sel]).mean(), it_c[sel].mean()
    print("seeded faces", int(sel.sum()), "mean iterations: plain", m_p, "learned", m_l,
          "converged-frame seed", m_c, "learned gain", m_p - m_l, "bound", m_p - 1.0, flush=True)
    assert np.all(it_c[sel] == 1)
    assert m_l >= m_c
    both = (it_p > 0) & (it_l > 0)
    du = np.abs(fr_l[both, :2] - fr_p[both, :2]).max(axis=1) / np.sqrt(fr_p[both, 2])
    dT = np.abs(fr_l[both, 2] - fr_p[both, 2]) / fr_p[both, 2]
    assert np.maximum(du, dT).max() <= 10 * tol
    torch.cuda.synchronize()
