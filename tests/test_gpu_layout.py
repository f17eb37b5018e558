"""The 2D state in its two layouts (pond_set_state_layout): the 12 Hermite coefficients per
cell (default) or the 32 populations themselves. They are a change of basis, exact on the
Gauss-Hermite nodes, so the step gives the same results in both to rounding: in FP64 the
parity bar of the finite-volume tests (1e-12 + 0.4 n tol after n steps), in the mixed form
relative L1 1e-6."""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu


def _relerr(a, b):
    out = []
    mom = np.abs(b[1:-1]).max()
    for k in range(b.shape[0]):
        scale = mom if 0 < k < b.shape[0] - 1 else np.abs(b[k]).max()
        out.append(np.abs(a[k] - b[k]).max() / (scale if scale > 0 else 1.0))
    return np.array(out)


def _print(tag, **kw):
    print(tag, " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def test_round_trip_keeps_the_populations():
    """Coefficients -> populations -> coefficients after 10 steps: the populations read out
    afterwards equal those before, to 1e-14 of their scale in FP64 and 1e-6 in the mixed
    form."""
    from paper_2203_05477_amd import pond

    cfg, f = W.double_mach(64, 32, tol=1e-12)
    for prec, bar in (("fp64", 1e-14), ("mixed", 1e-6)):
        g = pond.Context(cfg, f, precision=prec)
        g.step(10)
        f0, g0, fr0 = g.populations()
        g.set_state_layout("populations")
        g.set_state_layout("hermite")
        f1, g1, fr1 = g.populations()
        _print("layout_round_trip", precision=prec, f=np.abs(f1 - f0).max() / np.abs(f0).max(),
               g=np.abs(g1 - g0).max() / np.abs(g0).max())
        assert np.abs(f1 - f0).max() <= bar * np.abs(f0).max()
        assert np.abs(g1 - g0).max() <= bar * np.abs(g0).max()
        assert np.array_equal(fr1, fr0)
        g.close()


@pytest.mark.parametrize("case", ["double_mach", "random_periodic"])
def test_fp64_step_in_both_layouts(case):
    """The same FP64 steps from the same state with the state held as coefficients and as
    populations, through the face kernel, the tail kernel and both cell kernels (the
    default split) and with the split off: conserved fields and face frames to the parity
    bar; the double Mach reflection on 96 x 48 cells (fixed, split and moving-shock sides),
    30 steps; random periodic fields on 37 x 29 cells, 12 steps."""
    from paper_2203_05477_amd import pond

    if case == "double_mach":
        cfg, f = W.double_mach(96, 48, tol=1e-13)
        n = 30
    else:
        cfg, f = W.random_smooth(2, 37, 29, seed=3, amp=0.2, cfl=0.4, tol=1e-13)
        n = 12
    for split in (None, 0):
        a = pond.Context(cfg, f, precision="fp64")
        b = pond.Context(cfg, f, precision="fp64")
        if split is not None:
            a.set_iter_split(split)
            b.set_iter_split(split)
        b.set_state_layout("populations")
        a.step(n)
        b.step(n)
        e = _relerr(b.conserved(), a.conserved())
        ff = np.abs(b.face_frames() - a.face_frames()).max() / np.abs(a.face_frames()).max()
        _print("layout_fp64", case=case, split=split, err=e.max(), frames=ff)
        bar = 1e-12 + 0.4 * n * cfg["tol"]
        assert e.max() <= bar
        assert ff <= bar
        assert np.array_equal(a.time(), b.time()) or abs(a.time()[0] - b.time()[0]) <= 1e-13 * a.time()[0]
        b.set_state_layout("hermite")
        fa, ga, _ = a.populations()
        fb, gb, _ = b.populations()
        assert np.abs(fb - fa).max() <= bar * np.abs(fa).max()
        a.close()
        b.close()


def test_mixed_step_in_both_layouts():
    """The mixed form (FP32 populations) on the double Mach reflection, 40 steps at tol 1e-5
    with the autotuned tiles: relative L1 between the layouts <= 1e-6 per conserved field."""
    from paper_2203_05477_amd import pond

    cfg, f = W.double_mach(128, 32, tol=1e-5)
    a = pond.Context(cfg, f, precision="mixed")
    b = pond.Context(cfg, f, precision="mixed")
    b.set_state_layout("populations")
    a.autotune()
    b.autotune()
    a.step(40)
    b.step(40)
    Ua, Ub = a.conserved(), b.conserved()
    l1 = np.abs(Ub - Ua).sum(axis=1) / np.abs(Ua).sum(axis=1)
    _print("layout_mixed", l1=l1)
    assert np.all(l1 <= 1e-6)
    a.close()
    b.close()


def test_population_layout_refusals(tmp_path):
    from paper_2203_05477_amd import pond

    cfg, f = W.double_mach(32, 16)
    g = pond.Context(cfg, f, precision="fp64")
    g.set_state_layout("populations")
    with pytest.raises(pond.PondError):
        g.populations()
    with pytest.raises(pond.PondError):
        g.save(tmp_path / "x.ckpt")
    g.set_state_layout("hermite")
    g.save(tmp_path / "x.ckpt")
    g.close()
    bad = [dict(cfg, limiter="minmod"), dict(cfg, regularization="eq"), dict(cfg, scheme="sl")]
    for c in bad:
        h = pond.Context(c, f, precision="fp64")
        with pytest.raises(pond.PondError):
            h.set_state_layout("populations")
        h.close()
    c1, f1 = W.shock_tube(50)
    h = pond.Context(c1, f1, precision="fp64")
    with pytest.raises(pond.PondError):
        h.set_state_layout("populations")
    h.close()
