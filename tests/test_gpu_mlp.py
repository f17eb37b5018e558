"""GPU tests of the seed network: BF16-MFMA forward and backward kernels against the FP64
reference (oracle/mlp.py) evaluated with the same BF16 roundings, training, features, and
the learned seed inside the step.

Tolerances: the kernels round weights, inputs and hidden activations to BF16 (8-bit
mantissa, relative spacing 2^-8 = 3.9e-3) and accumulate in FP32; the reference applies
the same roundings in FP64, so the outputs agree to a few BF16 ulps where an activation
sits near a rounding boundary: relative norm error <= 1e-2 (forward) and <= 3e-2 (gradient,
which also rounds dZ to BF16 before the weight-gradient MFMAs).
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


def test_forward_matches_reference():
    import torch

    from oracle import mlp as M
    from paper_2203_05477_amd import pond

    p = M.he_params(5).astype(np.float32)
    p[M.NPARAM - 3:] = [0.1, -0.2, 0.3]
    net = pond.Mlp(params=p)
    for n in (1, 16, 37, 1000):
        X, _ = _data(n, n)
        Xd = torch.from_numpy(X).cuda()
        Yd = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        net.forward(Xd.data_ptr(), n, Yd.data_ptr())
        y = Yd.cpu().numpy()[:, :3]
        ref, _ = M.forward(p, X, bf16=True)
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        print("forward", n, err, flush=True)
        assert err <= 1e-2
        assert np.all(Yd.cpu().numpy()[:, 3] == 0.0)


def test_gradient_matches_reference():
    import torch

    from oracle import mlp as M
    from paper_2203_05477_amd import pond

    p = M.he_params(7).astype(np.float32)
    net = pond.Mlp(params=p)
    for n in (32, 50, 4096):
        X, T = _data(n, 100 + n)
        Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
        torch.cuda.synchronize()
        g, loss = net.grad(Xd.data_ptr(), Td.data_ptr(), n)
        lref, gref = M.loss_and_grad(p, X, T, bf16=True)
        err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
        print("grad", n, err, loss, lref, flush=True)
        assert err <= 3e-2
        assert loss == pytest.approx(lref, rel=1e-2)


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


def test_learned_seed_in_the_step():
    """Train on frames from a small double Mach run, then seed the same problem with the
    network: conservation stays exact and the result agrees with the plain run to the
    level that the iteration tolerance and the fallback faces allow."""
    import torch

    from paper_2203_05477_amd import learned_seed as LS
    from paper_2203_05477_amd import pond

    cfg, f = W.double_mach(192, 48, tol=1e-10)
    data = LS.harvest(cfg, f, steps=60, precision="fp64", hard_iters=2)
    net, losses, n = LS.train([data], epochs=20, batch=1024, lr=2e-3)
    print("samples", n, "loss", losses[0], losses[-1], flush=True)
    assert losses[-1] < losses[0]
    plain = pond.Context(cfg, f, precision="fp64")
    learned = pond.Context(cfg, f, precision="fp64", seed="mlp")
    learned.load_mlp(net, hard_iters=2)
    U0 = learned.conserved().sum(axis=1)
    sp = plain.step(80)
    sl = learned.step(80)
    print("iters plain", sp["iters_total"] / sp["faces"], "learned", sl["iters_total"] / sl["faces"],
          "nonconv", sp["nonconverged"], sl["nonconverged"], flush=True)
    Up, Ul = plain.conserved(), learned.conserved()
    l1 = np.abs(Ul - Up).sum(axis=1) / np.abs(Up).sum(axis=1)
    print("rel L1 learned vs plain", l1, flush=True)
    assert np.all(l1 < 1e-3)
    torch.cuda.synchronize()
