"""The end-of-call summary of pond_stats (smallest density and temperature, conserved
totals, first failing instance and cell, first non-converged face) and the per-call error
status, through the C ABI, against the read-outs of the same context and the FP64 oracle."""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_summary_matches_the_read_outs(orc):
    """Periodic random 2D field, FP64: totals = sum of U times dx dy (the totals of a
    periodic domain are also conserved, Sec. III.B), minima of the read-out fields, no
    failure, the first non-converged face as in pond_face_iters."""
    from paper_2203_05477_amd import pond

    cfg, f = W.random_smooth(2, 37, 29, seed=3, amp=0.4, tol=1e-13, max_iter=3)
    print("case random_smooth 37x29 max_iter 3", flush=True)
    g = pond.Context(cfg, f, precision="fp64")
    o = orc.Sim(cfg, f["rho"], f["ux"], f["uy"], f["p"])
    dv = (cfg["x1"] - cfg["x0"]) / cfg["nx"] * (cfg["y1"] - cfg["y0"]) / cfg["ny"]
    U0 = o.conserved().sum(axis=1) * dv
    for _ in range(4):
        st = g.step(1, check=False)
        o.step()
        U = g.conserved()
        tot = U.sum(axis=1) * dv
        assert np.allclose(st["totals"][:4], tot, rtol=1e-13, atol=1e-15)
        assert np.allclose(st["totals"][:4], U0, rtol=1e-13, atol=1e-14)
        r, _, _, T = g.moments()
        assert st["rho_min"] == r.min() and st["T_min"] == T.min()
        assert st["first_failed_instance"] == -1 and st["first_failed_cell"] == -1
        it = g.face_iters()
        bad = np.nonzero(it < 0)[0]
        assert st["first_nonconv_face"] == (int(bad[0]) if bad.size else -1)
        assert st["nonconverged"] == bad.size
    g.close()


def test_failure_reported_once_then_frozen(orc):
    """Double rarefaction on 800 cells (a known departure from Sec. IV.B: the step loses
    positivity next to the centre): the call whose step produced the invalid cell returns
    POND_ENONPHYS and names the instance and the lowest invalid cell (the oracle's first
    T <= 0 cell); the next call returns POND_OK with the instance still frozen."""
    from paper_2203_05477_amd import pond

    cfg, f = W.riemann_case("double_rarefaction", nx=800)
    print("case double_rarefaction 800", flush=True)
    g = pond.Context(cfg, f, precision="fp64")
    o = orc.Sim(cfg, f["rho"], f["ux"], None, f["p"])
    for n in range(1, 51):
        o.step(cfg["t_end"])
        st = g.step(1, cfg["t_end"], check=False)
        To = o.fields()[3]
        if not (To.min() > 0):
            assert st["status"] == pond.ENONPHYS
            assert st["first_failed_instance"] == 0 and st["failed_instances"] == 1
            assert st["first_failed_cell"] == int(np.nonzero(~(To > 0))[0][0])
            assert st["T_min"] <= 0.0
            break
        assert st["status"] == pond.OK and st["first_failed_cell"] == -1
    else:
        pytest.fail("the double rarefaction did not fail within 50 steps")
    t = g.time()[0]
    st = g.step(3, cfg["t_end"], check=False)
    assert st["status"] == pond.OK
    assert st["failed_instances"] == 1 and st["first_failed_instance"] == -1
    assert g.time()[0] == t
    g.close()


def test_first_failed_instance_of_a_batch(orc):
    """A batch of three tubes whose middle one is the double rarefaction: that instance is
    named when it fails, the two shock tubes go on, and the status of later calls is OK."""
    from paper_2203_05477_amd import pond

    parts = [W.shock_tube(96), W.riemann_case("double_rarefaction", nx=128), W.shock_tube(64)]
    cfg = dict(parts[0][0])
    cfg["lengths"] = [p[0]["nx"] for p in parts]
    cfg["nx"] = sum(cfg["lengths"])
    cfg["cfl"] = 0.2
    fields = {k: np.concatenate([p[1][k] for p in parts]) for k in ("rho", "ux", "p")}
    fields["uy"] = None
    print("case batch shock|double_rarefaction|shock", flush=True)
    g = pond.Context(cfg, fields, precision="fp64")
    seen = None
    for n in range(1, 200):
        st = g.step(1, check=False)
        if st["status"] == pond.ENONPHYS:
            seen = n
            assert st["first_failed_instance"] == 1
            assert 96 <= st["first_failed_cell"] < 96 + 128
            break
        assert st["status"] == pond.OK
    assert seen is not None
    t = g.time()
    st = g.step(5, check=False)
    assert st["status"] == pond.OK and st["failed_instances"] == 1
    t2 = g.time()
    assert t2[1] == t[1] and t2[0] > t[0] and t2[2] > t[2]
    assert np.array_equal(g.failed_instances(), np.array([0, 1, 0], dtype=np.int32))
    g.close()
