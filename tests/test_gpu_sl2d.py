"""GPU parity of the semi-Lagrangian realization in two dimensions (Sec. III.A on the D2Q16
lattice, POND_FLAG_SEMI_LAGRANGIAN) against the FP64 oracle, element by element.

Bars (FP64): relative max-norm error per conserved field <= 1e-12 + 0.4 n tol after n
steps, as for the 1D scheme (each cell's frame iteration stops within tol of its fixed
point, on each side in its own rounding); the populations of the next step to the same
bar. Grids are ragged: no side a multiple of the 16 x 16 cells of a block, and more than
one block along each axis, so partly filled blocks and the LDS tiles' seams are covered.
At full size (1920 x 480), where the oracle is too slow, the closed form of an affine
density (the explicit Euler update, exact for the scheme) is checked on every cell."""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sl(cfg):
    return dict(cfg, scheme="sl")


def _relerr(a, b):
    out = []
    mom = np.abs(b[1:-1]).max()
    for k in range(b.shape[0]):
        scale = mom if 0 < k < b.shape[0] - 1 else np.abs(b[k]).max()
        out.append(np.abs(a[k] - b[k]).max() / (scale if scale > 0 else 1.0))
    return np.array(out)


def _print(tag, **kw):
    print(tag, " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _pair(orc, cfg, f, precision="fp64"):
    from paper_2203_05477_amd import pond

    cfg = _sl(cfg)
    return pond.Context(cfg, f, precision=precision), orc.Sim(cfg, f["rho"], f["ux"], f["uy"], f["p"])


def _bar(n, tol):
    return 1e-12 + 0.4 * n * tol


@pytest.mark.parametrize("reg", ["grad", "eq"])
def test_random_periodic_fp64(orc, reg):
    """Smooth random fields on a periodic 37 x 21 grid (3 x 2 blocks), 6 steps: conserved
    fields, clock, iteration totals, and the populations the next step starts from (all
    16 of f and of g in each cell's frame); both regularizations of f."""
    cfg, f = W.random_smooth(2, 37, 21, seed=7, amp=0.25, cfl=0.4, tol=1e-13)
    if reg == "eq":
        cfg["regularization"] = "eq"
    _print("case", name="sl2d_random", reg=reg)
    g, o = _pair(orc, cfg, f)
    it_g = it_o = 0
    for k in range(6):
        o.step()
        st = g.step(1)
        it_g += st["iters_total"]
        it_o += o.last["iters_total"]
        e = _relerr(g.conserved(), o.conserved())
        assert e.max() <= _bar(k + 1, cfg["tol"]), (k, e)
    _print("sl2d_random", reg=reg, err=e.max(), iters_gpu=it_g, iters_oracle=it_o)
    assert g.time()[0] == pytest.approx(o.t, rel=1e-13)
    assert abs(it_g - it_o) <= 0.01 * it_o
    fg, gg, frg = g.populations()
    fo, go, fro = o.reframed()
    assert np.abs(fg - fo).max() <= _bar(6, cfg["tol"]) * np.abs(fo).max()
    assert np.abs(gg - go).max() <= _bar(6, cfg["tol"]) * np.abs(go).max()
    assert np.abs(frg - fro).max() <= _bar(6, cfg["tol"]) * np.abs(fro).max()
    g.close()


def test_mixed_sides_fp64(orc):
    """Outflow sides along x and reflecting sides along y (mirrored ghosts in the tiles of
    the first and last block rows and columns), 33 x 19 cells, 8 steps."""
    cfg, f = W.random_smooth(2, 33, 19, seed=11, amp=0.2, cfl=0.4, tol=1e-13)
    cfg["bc"] = ["outflow", "outflow", "reflect", "reflect"]
    _print("case", name="sl2d_sides")
    g, o = _pair(orc, cfg, f)
    for k in range(8):
        o.step()
        g.step(1)
        e = _relerr(g.conserved(), o.conserved())
        assert e.max() <= _bar(k + 1, cfg["tol"]), (k, e)
    _print("sl2d_sides", err=e.max())
    g.close()


@pytest.mark.parametrize("axis", [0, 1])
def test_sod_along_each_axis_fp64(orc, axis):
    """Sod's problem along x or along y (70 cells along, 3 periodic cells across), 60 steps:
    the shock, the contact and the rarefaction through the clip."""
    n, nt = 70, 3
    nx, ny = (n, nt) if axis == 0 else (nt, n)
    bc = ("outflow", "outflow", "periodic", "periodic") if axis == 0 else ("periodic", "periodic", "outflow", "outflow")
    cfg = W.base_config(2, nx, ny, cfl=0.4, tol=1e-13, bc=bc)
    X, Y = W.cell_centres(cfg)
    left = (X if axis == 0 else Y) < 0.5
    f = {"rho": np.where(left, 1.0, 0.125), "ux": np.zeros_like(X), "uy": np.zeros_like(X),
         "p": np.where(left, 1.0, 0.1)}
    _print("case", name="sl2d_sod", axis=axis)
    g, o = _pair(orc, cfg, f)
    for k in range(60):
        o.step()
        g.step(1)
    e = _relerr(g.conserved(), o.conserved())
    _print("sl2d_sod", axis=axis, err=e.max())
    assert e.max() <= _bar(60, cfg["tol"])
    g.close()


def test_double_mach_small_fp64(orc):
    """The double Mach reflection on 96 x 24 cells (fixed inflow, the moving-shock top side,
    the split bottom side), 30 steps at tol 1e-12 with up to 64 iterations per cell (one
    cell of step 7 takes 57; four cells of step 2 stop at a 2-cycle)."""
    cfg, f = W.double_mach(96, 24, tol=1e-12, max_iter=64)
    _print("case", name="sl2d_dmr")
    g, o = _pair(orc, cfg, f)
    for k in range(30):
        o.step()
        g.step(1)
    e = _relerr(g.conserved(), o.conserved())
    _print("sl2d_dmr", err=e.max())
    assert e.max() <= _bar(30, cfg["tol"])
    assert g.time()[0] == pytest.approx(o.t, rel=1e-13)
    g.close()


def test_mixed_precision_against_the_oracle(orc):
    """The mixed form (FP32 populations, FP64 conserved variables) at tol 1e-5 against the
    FP64 oracle at the same tolerance: relative L1 <= 1e-4 per conserved field after 20
    steps of the shocked interface on 64 x 16 cells."""
    cfg, f = W.shocked_interface(64, 16, tol=1e-5)
    g, o = _pair(orc, cfg, f, precision="mixed")
    for _ in range(20):
        o.step()
        g.step(1)
    Ug, Uo = g.conserved(), o.conserved()
    l1 = np.abs(Ug - Uo).sum(axis=1) / np.maximum(np.abs(Uo).sum(axis=1), 1e-300)
    _print("sl2d_mixed", l1=l1)
    assert l1[0] < 1e-4 and l1[1] < 1e-4 and l1[3] < 1e-4


def test_uniform_state_is_kept():
    from paper_2203_05477_amd import pond

    cfg, f = W.uniform(2, 35, 18, rho=1.3, u=(0.3, -0.45), p=0.7, tol=1e-13)
    for prec, bar in (("fp64", 1e-13), ("mixed", 2e-6)):
        g = pond.Context(_sl(cfg), f, precision=prec)
        g.step(5)
        U = g.conserved()
        ref = np.array([1.3, 1.3 * 0.3, -1.3 * 0.45, 0.7 / 0.4 + 0.5 * 1.3 * (0.09 + 0.2025)])
        assert np.abs(U - ref[:, None]).max() <= bar * np.abs(ref).max(), prec
        g.close()


def _affine(nx, ny, u, T=0.8, gx=0.3, gy=0.2, tol=1e-13):
    cfg = W.base_config(2, nx, ny, cfl=0.3, tol=tol, mu=1e-3, bc=("outflow",) * 4)
    X, Y = W.cell_centres(cfg)
    rho = 1.0 + gx * X + gy * Y
    f = {"rho": rho, "ux": np.full_like(X, u[0]), "uy": np.full_like(X, u[1]), "p": rho * T}
    return cfg, f


def _affine_expected(cfg, U0, dt, u, T=0.8, gx=0.3, gy=0.2):
    Cv = 1.0 / (cfg["gamma"] - 1.0)
    ug = u[0] * gx + u[1] * gy
    return np.stack([U0[0] - dt * ug, U0[1] - dt * (ug * u[0] + T * gx), U0[2] - dt * (ug * u[1] + T * gy),
                     U0[3] - dt * ug * (0.5 * (u[0] ** 2 + u[1] ** 2) + (Cv + 1.0) * T)])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_affine_density_closed_form(precision):
    """1920 x 480 cells (the double Mach grid), an affine density in a uniform flow at
    uniform temperature, one step in the bench's launch shape: every cell two or more cells
    from the sides holds the explicit Euler update U - dt div F(U) (exact for the scheme:
    the cubic kernel reproduces affine populations and the clip does not act on them).
    FP64 to 1e-12 relative; mixed to 1e-5 (FP32 populations, and at tol 1e-6 the
    collision keeps momentum to about rho tol sqrt(T))."""
    from paper_2203_05477_amd import pond

    nx, ny, u = 1920, 480, (0.6, -0.35)
    cfg, f = _affine(nx, ny, u, tol=1e-13 if precision == "fp64" else 1e-6)
    _print("case", name="sl2d_affine_full", precision=precision)
    g = pond.Context(_sl(cfg), f, precision=precision)
    U0 = g.conserved()
    g.step(1)
    dt = g.time()[0]
    ex = _affine_expected(cfg, U0, dt, u)
    U = g.conserved()
    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    inner = ((I >= 2) & (I < nx - 2) & (J >= 2) & (J < ny - 2)).ravel()
    err = np.abs(U[:, inner] - ex[:, inner]).max(axis=1) / np.abs(ex[:, inner]).max(axis=1).clip(1.0)
    _print("sl2d_affine_full", precision=precision, err=err)
    assert np.all(err <= (1e-12 if precision == "fp64" else 1e-5)), err
    g.close()


def test_graph_replay_and_resume_are_bitwise(tmp_path):
    """Steps replayed from a captured HIP graph, and a run resumed from a checkpoint, give
    the bits of the launched steps."""
    from paper_2203_05477_amd import pond

    cfg, f = W.random_smooth(2, 40, 20, seed=4, cfl=0.4, tol=1e-12)
    a = pond.Context(_sl(cfg), f, precision="fp64")
    a.step(3)
    path = tmp_path / "sl2d.ckpt"
    a.save(path)
    a.step(6)
    b = pond.Context(_sl(cfg), f, precision="fp64")
    b.load_state(path)
    b.set_graph(True)
    b.step(6)
    assert np.array_equal(a.conserved(), b.conserved())
    assert np.array_equal(a.time(), b.time())
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_iteration_split_gives_the_same_state(precision):
    """Cells still iterating after k iterations finish in the tail kernel, which builds the
    stencil records from the state instead of the LDS tile and continues the same
    iteration from the saved frames: k = 1 (nearly every cell of this case goes to the
    tail: about 4 iterations per cell), k = 3 and the default give the state of k = 0 (no
    tail) to rounding: the tail sums each population over the stencil in another order, so
    a frame may stop one iteration apart at the tolerance (FP64: the parity bar, 1e-12 +
    0.4 n tol after n steps; the mixed form at tol 1e-4: 1e-5), with iteration totals
    within 1%."""
    from paper_2203_05477_amd import pond

    tol = 1e-13 if precision == "fp64" else 1e-4
    cfg, f = W.random_smooth(2, 37, 21, seed=7, amp=0.25, cfl=0.4, tol=tol)
    out = {}
    for k in (0, 1, 3, None):
        g = pond.Context(_sl(cfg), f, precision=precision)
        if k is not None:
            g.set_iter_split(k)
        st = g.step(5)
        out[k] = (g.conserved(), st["iters_total"], st["cell_updates"])
        g.close()
    bar = _bar(5, tol) if precision == "fp64" else 1e-5
    for k in (1, 3, None):
        e = _relerr(out[k][0], out[0][0])
        _print("sl2d_split", precision=precision, k=k, err=e.max(), iters=out[k][1], iters_nosplit=out[0][1])
        assert e.max() <= bar, (k, e)
        assert out[k][2] == out[0][2]
        assert abs(out[k][1] - out[0][1]) <= 0.01 * out[0][1], k
