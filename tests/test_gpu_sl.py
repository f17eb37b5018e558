"""GPU parity of the semi-Lagrangian realization (Sec. III.A, 1D; POND_FLAG_SEMI_LAGRANGIAN)
against the FP64 oracle. Over thousands of steps the iteration tolerance bounds the
agreement, as for the finite-volume Riemann runs: bar 1e-12 + 0.4 n tol after n steps."""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sl(cfg):
    return dict(cfg, scheme="sl")


def _relerr(a, b):
    return np.array([np.abs(a[k] - b[k]).max() / max(np.abs(b[k]).max(), 1e-300)
                     for k in range(b.shape[0])])


@pytest.mark.parametrize("case", ["shock_tube", "lax"])
def test_sl_fp64_parity(orc, case):
    """400 cells to the final time: conserved fields against the oracle every 50 steps and
    at the end, the same final time."""
    from paper_2203_05477_amd import pond

    if case == "shock_tube":
        cfg, f = W.shock_tube(400)
    else:
        cfg, f = W.riemann_case("lax", nx=400)
    cfg = _sl(cfg)
    t_end = cfg["t_end"]
    print("case sl", case, flush=True)
    g = pond.Context(cfg, f, precision="fp64")
    o = orc.Sim(cfg, f["rho"], f["ux"], None, f["p"])
    n = 0
    while o.t < t_end * (1 - 1e-12):
        o.step(t_end)
        g.step(1, t_end)
        n += 1
        if n % 50 == 0:
            e = _relerr(g.conserved(), o.conserved())
            assert e.max() <= 1e-12 + 0.4 * n * cfg["tol"], (n, e)
    assert g.time()[0] == pytest.approx(o.t, rel=1e-13)
    e = _relerr(g.conserved(), o.conserved())
    print("sl", case, "steps", n, "err", e.max(), flush=True)
    assert e.max() <= 1e-12 + 0.4 * n * cfg["tol"]
    g.close()


def test_sl_tube_batch_parity(orc):
    """A batch of uneven tubes (20..120 cells) in one context: each tube against its own
    oracle run, 20 steps."""
    from paper_2203_05477_amd import pond

    batch, fields = W.tube_batch(n_tubes=12, len_lo=20, len_hi=120, tol=1e-13, rho_decades=1.0,
                                 p_decades=1.0, mach=1.0)
    batch = _sl(batch)
    print("case sl tubes", flush=True)
    g = pond.Context(batch, fields, precision="fp64")
    g.step(20, check=False)
    U = g.conserved()
    off = np.concatenate([[0], np.cumsum(batch["lengths"])])
    worst = 0.0
    for k in range(len(batch["lengths"])):
        c = _sl(W.tube_config(batch, k))
        ff = W.tube_fields(batch, fields, k)
        o = orc.Sim(c, ff["rho"], ff["ux"], None, ff["p"])
        for _ in range(20):
            o.step()
        Uo = o.conserved()
        sl = slice(off[k], off[k + 1])
        worst = max(worst, _relerr(U[:, sl], Uo).max())
    print("sl tubes err", worst, flush=True)
    assert worst <= 1e-12
    g.close()


def test_sl_mixed_close_to_fp64_and_flags():
    """The mixed form tracks the FP64 form on the shock tube; the resident launch is
    refused with the scheme."""
    from paper_2203_05477_amd import pond

    out = {}
    for prec, tol in (("fp64", W.TOL_FP64), ("mixed", W.TOL_FP32)):
        cfg, f = W.shock_tube(400, tol=tol)
        g = pond.Context(_sl(cfg), f, precision=prec)
        g.step(1000, 0.2)
        assert g.time()[0] == pytest.approx(0.2, rel=1e-13)
        out[prec] = g.conserved()
        if prec == "fp64":
            with pytest.raises(pond.PondError):
                g.set_resident(True)
        g.close()
    d = np.abs(out["mixed"] - out["fp64"]).sum(axis=1) / np.abs(out["fp64"]).sum(axis=1)
    print("sl mixed vs fp64", d, flush=True)
    assert np.all(d < 1e-4)
