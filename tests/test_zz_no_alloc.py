"""pond_mlp_train_noalloc (the training entry point for callers that cannot allocate)
against pond_mlp_train, through the C ABI: two networks with the same initial weights
trained on the same data give the same epoch losses and parameters bit for bit, on two
calls in a row (the second with fewer samples, so the static buffer holds a longer
previous call's losses), and sizes beyond the static buffer are refused with the network
unchanged."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _data(torch, n, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.zeros(n, 64, dtype=torch.float32)
    X[:, :40] = torch.randn(n, 40, generator=g) * 0.5
    T = torch.zeros(n, 4, dtype=torch.float32)
    T[:, :3] = torch.tanh(X[:, :3] * 0.7 + 0.1 * X[:, 3:6])
    return X.cuda(), T.cuda()


def test_noalloc_training_matches_the_allocating_entry_point():
    import torch

    from paper_2203_05477_amd import pond

    a = pond.Mlp(seed=5)
    b = pond.Mlp(seed=5)
    assert np.array_equal(a.params(), b.params())
    for call, (n, epochs, batch) in enumerate(((3000, 3, 256), (700, 2, 64))):
        X, T = _data(torch, n, seed=11 + call)
        print("noalloc call", call, "n", n, "epochs", epochs, "batch", batch, flush=True)
        la = a.train(X.data_ptr(), T.data_ptr(), n, epochs=epochs, batch=batch, lr=2e-3)
        lb = b.train_noalloc(X.data_ptr(), T.data_ptr(), n, epochs=epochs, batch=batch, lr=2e-3)
        torch.cuda.synchronize()
        print("losses", la, lb, flush=True)
        assert np.array_equal(la, lb)
        assert np.array_equal(a.params(), b.params())
    a.close()
    b.close()


def test_noalloc_refuses_sizes_beyond_its_buffer():
    import torch

    from paper_2203_05477_amd import pond

    m = pond.Mlp(seed=2)
    p0 = m.params()
    # one more batch per epoch than the static buffer holds (real arrays of that size, so
    # nothing could read past them even if the check were missing)
    n = (65536 + 1) * 32
    X = torch.zeros(n, 64, dtype=torch.float32, device="cuda")
    T = torch.zeros(n, 4, dtype=torch.float32, device="cuda")
    print("noalloc refusal n", n, flush=True)
    with pytest.raises(pond.PondError) as e:
        m.train_noalloc(X.data_ptr(), T.data_ptr(), n, epochs=1, batch=32)
    assert e.value.status == pond.EINVAL
    with pytest.raises(pond.PondError) as e:
        m.train_noalloc(X.data_ptr(), T.data_ptr(), 64, epochs=4097, batch=32)
    assert e.value.status == pond.EINVAL
    assert np.array_equal(m.params(), p0)
    m.close()
