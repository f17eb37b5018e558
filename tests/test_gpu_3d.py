"""GPU parity of the three-dimensional step (D3Q64 lattice, 20-moment Grad projection)
through the C ABI, against the FP64 oracle element by element.

Tolerance (FP64): relative max-norm error <= 1e-12 per conserved field after the same steps
from the same state, both sides iterating the face frames to the same tolerance; face
moments and frames <= 1e-11 of their scale; face iteration counts equal on >= 99% of the
faces (a face whose last frame change sits at the tolerance may take one iteration more on
one side). The random fields keep every face's iteration well inside max_iter (at larger
amplitudes some faces need 30-45 iterations to reach 1e-13, and a face that converges
exactly at the cap on one side and not on the other takes a different state). Grid sizes
are ragged (no axis a multiple of the four lanes per face or of the
256-thread blocks), so partly filled waves and blocks are covered."""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _pair(orc, cfg, f, precision="fp64"):
    from paper_2203_05477_amd import pond

    g = pond.Context(cfg, f, precision=precision)
    o = orc.Sim(cfg, f["rho"], f["ux"], f["uy"], f["p"], uz=f["uz"])
    return g, o


def _relerr(a, b):
    """Max-norm error per conserved field relative to its largest value (the momentum
    components share the scale of the momentum vector)."""
    out = []
    mom = np.abs(b[1:-1]).max()
    for k in range(b.shape[0]):
        scale = mom if 0 < k < b.shape[0] - 1 else np.abs(b[k]).max()
        out.append(np.abs(a[k] - b[k]).max() / (scale if scale > 0 else 1.0))
    return np.array(out)


def _print(tag, **kw):
    print(tag, " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def test_random_periodic_fp64(orc):
    """Smooth random fields in a periodic 9 x 7 x 6 box, 4 steps: conserved fields, clocks,
    face moments (lab frame), face frames, iteration counts, and the populations the next
    step starts from (all 64 of f and of g in each cell's frame). At most 24 iterations per
    face in the oracle."""
    cfg, f = W.random_smooth_3d(9, 7, 6, seed=5, cfl=0.3, tol=1e-13, amp=0.2)
    _print("case", name="random3d", shape=(9, 7, 6))
    g, o = _pair(orc, cfg, f)
    for _ in range(4):
        o.step()
        g.step(1)
    assert g.time()[0] == pytest.approx(o.t, rel=1e-13)
    e = _relerr(g.conserved(), o.conserved())
    _print("random3d", err=e.max())
    assert e.max() <= TOL64
    Mf_g, Mg_g = g.face_moments()
    Mf_o, Mg_o = o.face_moments()
    assert np.abs(Mf_g - Mf_o).max() <= 1e-11 * np.abs(Mf_o).max()
    assert np.abs(Mg_g - Mg_o).max() <= 1e-11 * np.abs(Mg_o).max()
    ff, fo = g.face_frames(), o.face_frames()
    assert np.abs(ff - fo).max() <= 1e-11 * np.abs(fo).max()
    it_g, it_o = g.face_iters(), o.face_iters()
    assert np.mean(np.abs(it_g) == np.abs(it_o)) > 0.99
    fg, gg, frg = g.populations()
    fo_, go_, fro = o.reframed()
    assert np.abs(fg - fo_).max() <= TOL64 * np.abs(fo_).max()
    assert np.abs(gg - go_).max() <= TOL64 * np.abs(go_).max()
    assert np.abs(frg - fro).max() <= TOL64 * np.abs(fro).max()


@pytest.mark.parametrize("limiter", ["vanleer", "minmod"])
def test_mixed_sides_fp64(orc, limiter):
    """Outflow sides along x, reflecting along y, periodic along z (every side kind on
    every axis position of the stencil: mirrored cells flip the normal velocity and the
    odd coefficients), 6 steps, both limiters (at most 28 iterations per face)."""
    cfg, f = W.random_smooth_3d(11, 6, 5, seed=9, cfl=0.3, tol=1e-13, amp=0.15)
    cfg["bc"] = ["outflow", "outflow", "reflect", "reflect", "periodic", "periodic"]
    cfg["limiter"] = limiter
    _print("case", name="sides3d", limiter=limiter)
    g, o = _pair(orc, cfg, f)
    for k in range(6):
        o.step()
        g.step(1)
        e = _relerr(g.conserved(), o.conserved())
        assert e.max() <= TOL64, (k, e)
    _print("sides3d", limiter=limiter, err=e.max())


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_riemann_problem_along_each_axis_fp64(orc, axis):
    """Sod's problem along x, y or z (3 periodic cells across, 70 cells along), 40 steps:
    a shock, a contact and a rarefaction crossing the faces of one axis."""
    cfg, f = W.riemann_3d((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), axis=axis, n=70, nt=3, tol=1e-13)
    _print("case", name="riemann3d", axis=axis)
    g, o = _pair(orc, cfg, f)
    for k in range(40):
        o.step()
        g.step(1)
    e = _relerr(g.conserved(), o.conserved())
    _print("riemann3d", axis=axis, err=e.max())
    assert e.max() <= TOL64
    assert g.time()[0] == pytest.approx(o.t, rel=1e-13)


EPS64 = 2.0 ** -52


def test_strong_shock_with_restarts_fp64(orc):
    """A temperature ratio of 1e5 along z (the strong shock tube's states, Sec. IV.B): the
    first steps take restarts from the mean frame and first-order fallbacks on both sides
    of the comparison; the fallback counts agree. Bar after n steps: 1e-12 + n eps T_max /
    T_min. The oracle writes the projection with lab-frame moments, as the paper does, and
    a hot cell projected into a face frame near the cold side's temperature subtracts
    second moments of size rho T_max to leave rho T_frame: it loses up to T_max / T_min of
    the 16 digits in that face state (the GPU's frame-relative shift does not)."""
    cfg, f = W.riemann_3d((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01), axis=2, n=60, nt=2, tol=1e-13,
                          cfl=0.2)
    _print("case", name="strong3d")
    g, o = _pair(orc, cfg, f)
    fb_g = fb_o = 0
    worst = 0.0
    for k in range(12):
        o.step()
        st = g.step(1)
        fb_g += st["fallback"]
        fb_o += o.last["nonphysical"]
        e = _relerr(g.conserved(), o.conserved())
        bar = 1e-12 + (k + 1) * EPS64 * 1e5
        worst = max(worst, e.max() / bar)
        assert e.max() <= bar, (k, e)
    _print("strong3d", err=e.max(), worst_err_over_bar=worst, fallback_gpu=fb_g, fallback_oracle=fb_o)
    assert fb_g == fb_o and fb_o > 0


def test_uniform_state_is_kept(orc):
    """A uniform moving state is a fixed point of the GPU step in both precisions."""
    from paper_2203_05477_amd import pond

    cfg = W.base_config_3d(7, 6, 5, tol=1e-13)
    n = 7 * 6 * 5
    f = {"rho": np.full(n, 1.3), "ux": np.full(n, 0.3), "uy": np.full(n, -0.2), "uz": np.full(n, 0.45),
         "p": np.full(n, 0.7)}
    for prec, bar in (("fp64", 1e-13), ("mixed", 1e-6)):
        g = pond.Context(cfg, f, precision=prec)
        g.step(5)
        U = g.conserved()
        ref = np.array([1.3, 1.3 * 0.3, -1.3 * 0.2, 1.3 * 0.45, 0.7 / (1.4 - 1) + 0.5 * 1.3 * (0.09 + 0.04 + 0.2025)])
        assert np.abs(U - ref[:, None]).max() <= bar * np.abs(ref).max(), prec


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_periodic_conservation(precision):
    """Mass, the three momenta and energy on a periodic box: the FP64 flux-form update of
    the conserved variables telescopes exactly between neighbours, so the totals hold to
    round-off in both precisions, and pond_stats' totals equal the sums of the read-out."""
    from paper_2203_05477_amd import pond

    cfg, f = W.random_smooth_3d(10, 9, 7, seed=2, cfl=0.3, tol=1e-5 if precision == "mixed" else 1e-12)
    g = pond.Context(cfg, f, precision=precision)
    vol = 1.0 / (10 * 9 * 7)
    U0 = g.conserved().sum(axis=1)
    st = g.step(8)
    U = g.conserved()
    scale = np.abs(U).sum(axis=1)
    assert np.all(np.abs(U.sum(axis=1) - U0) <= 1e-13 * scale)
    tot = np.array(st["totals"])
    assert np.all(np.abs(tot - U.sum(axis=1) * vol) <= 1e-13 * scale * vol)
    assert st["faces"] == 8 * g.nfaces and st["cell_updates"] == 8 * 630


def test_mixed_precision_against_the_oracle(orc):
    """The mixed form (FP32 populations, FP64 conserved variables) at iteration tolerance
    1e-5 against the FP64 oracle at the same tolerance: relative L1 <= 1e-4 per conserved
    field after 10 steps of the Sod problem along y."""
    cfg, f = W.riemann_3d((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), axis=1, n=64, nt=3, tol=1e-5)
    g, o = _pair(orc, cfg, f, precision="mixed")
    for _ in range(10):
        o.step()
        g.step(1)
    Ug, Uo = g.conserved(), o.conserved()
    l1 = np.abs(Ug - Uo).sum(axis=1) / np.maximum(np.abs(Uo).sum(axis=1), 1e-300)
    _print("mixed3d", l1=l1)
    assert l1[0] < 1e-4 and l1[2] < 1e-4 and l1[4] < 1e-4


def test_graph_replay_and_resume_are_bitwise(tmp_path):
    """Steps replayed from a captured HIP graph, and a run resumed from a checkpoint, give
    the bits of the launched steps."""
    from paper_2203_05477_amd import pond

    cfg, f = W.random_smooth_3d(8, 7, 6, seed=4, cfl=0.3, tol=1e-12)
    a = pond.Context(cfg, f, precision="fp64")
    a.step(3)
    path = tmp_path / "s3.ckpt"
    a.save(path)
    a.step(6)
    b = pond.Context(cfg, f, precision="fp64")
    b.load_state(path)
    b.set_graph(True)
    b.step(6)
    assert np.array_equal(a.conserved(), b.conserved())
    assert np.array_equal(a.face_frames(), b.face_frames())
    assert np.array_equal(a.time(), b.time())


def test_invalid_3d_configurations_are_rejected():
    from paper_2203_05477_amd import pond

    cfg, f = W.random_smooth_3d(6, 5, 4, seed=1)
    cfg1, f1 = W.random_smooth_3d(6, 5, 1, seed=1)  # one cell along z
    bad = [(dict(cfg, bc=["fixed"] + cfg["bc"][1:]), f),          # a kind 3D does not take
           (cfg1, f1),
           (dict(cfg, gamma=1.8), f),                               # C_v < 3/2
           (dict(cfg, regularization="eq"), f),                     # Grad projection only
           (dict(cfg, bc=cfg["bc"][:4] + ["periodic", "outflow"]), f)]  # unpaired periodic side
    for c, ff in bad:
        with pytest.raises(pond.PondError):
            pond.Context(c, ff, precision="fp64")
    g = pond.Context(cfg, f, precision="fp64")
    with pytest.raises(pond.PondError):
        g.set_tiles(16, 16)
    with pytest.raises(pond.PondError):
        g.set_resident(True)
