"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by element.

Tolerance (FP64): relative max-norm error <= 1e-12 per conserved field, the bar stated for
the FP64 form; both sides iterate the face frames to tol = 1e-13 from the same seeds.
"""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _pair(orc, cfg, f, precision="fp64"):
    from paper_2203_05477_amd import pond

    g = pond.Context(cfg, f, precision=precision)
    o = orc.Sim(cfg, f["rho"], f["ux"], f.get("uy"), f["p"])
    return g, o


def _relerr(a, b):
    """Max-norm error per conserved field, relative to the field's largest value; the
    momentum components share the scale of the momentum vector (a component that is zero
    up to round-off, e.g. rho u_y of a symmetric flow, is not judged against itself)."""
    out = []
    mom = np.abs(b[1:-1]).max()
    for k in range(b.shape[0]):
        scale = mom if 0 < k < b.shape[0] - 1 else np.abs(b[k]).max()
        out.append(np.abs(a[k] - b[k]).max() / (scale if scale > 0 else 1.0))
    return np.array(out)


def _print(tag, **kw):
    print(tag, " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def test_shock_tube_full_run_fp64(orc):
    """The 400-cell shock tube to t = 0.2 at CFL 0.5 (about 540 steps): conserved fields,
    face frames and the populations the next step starts from."""
    cfg, f = W.shock_tube(400)
    _print("case", name="shock_tube", n=400)
    g, o = _pair(orc, cfg, f)
    n = 0
    while o.t < 0.2 * (1 - 1e-14):
        o.step(0.2)
        g.step(1, 0.2)
        n += 1
    assert g.time()[0] == pytest.approx(o.t, rel=1e-13)
    e = _relerr(g.conserved(), o.conserved())
    _print("shock_tube", steps=n, err=e.max())
    assert e.max() <= TOL64
    fg, gg, frg = g.populations()
    fo, go, fro = o.reframed()
    assert np.abs(fg - fo).max() <= TOL64 * np.abs(fo).max()
    assert np.abs(gg - go).max() <= TOL64 * np.abs(go).max()
    assert np.abs(frg - fro).max() <= TOL64 * np.abs(fro).max()
    ff = g.face_frames()
    fo2 = o.face_frames()
    assert np.abs(ff - fo2).max() <= 1e-11 * np.abs(fo2).max()


@pytest.mark.parametrize("nx,ny,steps", [(40, 24, 8), (67, 35, 4)])
def test_periodic_random_2d_fp64(orc, nx, ny, steps):
    """Smooth random periodic fields on ragged grid sizes (several LDS tiles and a tail)."""
    cfg, f = W.random_smooth(2, nx, ny, seed=7, cfl=0.3, tol=1e-13)
    _print("case", name="random2d", nx=nx, ny=ny)
    g, o = _pair(orc, cfg, f)
    for _ in range(steps):
        o.step()
        g.step(1)
    e = _relerr(g.conserved(), o.conserved())
    _print("random2d", err=e.max())
    assert e.max() <= TOL64
    Mf_g, Mg_g = g.face_moments()
    Mf_o, Mg_o = o.face_moments()
    assert np.abs(Mf_g - Mf_o).max() <= 1e-11 * np.abs(Mf_o).max()
    assert np.abs(Mg_g - Mg_o).max() <= 1e-11 * np.abs(Mg_o).max()
    it_g, it_o = g.face_iters(), o.face_iters()
    assert np.mean(np.abs(it_g) == np.abs(it_o)) > 0.99


@pytest.mark.parametrize("split", [None, 0, 1])
def test_double_mach_small_fp64(orc, split):
    """Double Mach reflection on 96 x 24 cells, 30 steps: fixed, split fixed/reflecting,
    moving-shock and outflow boundaries, strong shocks, restarts and fallbacks. With the
    default hand-over to the tail kernel, without tail kernel (split 0), and with every
    iteration after the first in the tail kernel (split 1)."""
    cfg, f = W.double_mach(96, 24)
    _print("case", name="dmr", nx=96, ny=24, split=split)
    g, o = _pair(orc, cfg, f)
    if split is not None:
        g.set_iter_split(split)
    for k in range(30):
        o.step()
        g.step(1)
        e = _relerr(g.conserved(), o.conserved())
        assert e.max() <= TOL64, (k, e)
    _print("dmr", err=e.max(), fallback=o.last["nonphysical"])


@pytest.mark.parametrize("dim", [1, 2])
def test_minmod_limiter_fp64(orc, dim):
    """The minmod limiter (a separate kernel instantiation): 1D shock tube and 2D double
    Mach reflection against the oracle."""
    if dim == 1:
        cfg, f = W.shock_tube(200)
        steps = 120
    else:
        cfg, f = W.double_mach(64, 16)
        steps = 20
    cfg["limiter"] = "minmod"
    _print("case", name="minmod", dim=dim)
    g, o = _pair(orc, cfg, f)
    for _ in range(steps):
        o.step()
        g.step(1)
    e = _relerr(g.conserved(), o.conserved())
    _print("minmod", dim=dim, err=e.max())
    assert e.max() <= TOL64


def test_uniform_state_is_kept_gpu(orc):
    from paper_2203_05477_amd import pond

    cfg, f = W.uniform(2, 33, 17, tol=1e-13)
    for prec, tol in (("fp64", 1e-13), ("mixed", 2e-6)):
        g = pond.Context(cfg, f, precision=prec)
        g.step(3)
        r, ux, uy, T = g.moments()
        assert np.abs(r - 1).max() < tol and np.abs(ux - 0.3).max() < tol
        assert np.abs(uy + 0.2).max() < tol and np.abs(T - 0.7).max() < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_periodic_conservation_gpu(orc, precision):
    """FP64 conserved update: totals exact to FP64 round-off in both precisions."""
    from paper_2203_05477_amd import pond

    cfg, f = W.random_smooth(2, 48, 32, seed=2, cfl=0.3, tol=1e-12 if precision == "fp64" else 1e-5)
    g = pond.Context(cfg, f, precision=precision)
    U0 = g.conserved().sum(axis=1)
    g.step(20)
    U1 = g.conserved().sum(axis=1)
    scale = np.abs(g.conserved()).sum(axis=1)
    assert np.all(np.abs(U1 - U0) <= 1e-13 * scale)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_periodic_conservation_with_tail(precision):
    """Periodic blast (dense, high-pressure square) with one face iteration per face kernel,
    so that many faces go to the tail and their stencil cells are updated after it by
    another kernel than the rest: the face fluxes still telescope, totals stay exact to FP64
    round-off."""
    from paper_2203_05477_amd import pond

    cfg, f = W.random_smooth(2, 64, 48, seed=5, amp=0.0, cfl=0.3,
                             tol=1e-12 if precision == "fp64" else 1e-5)
    X, Y = W.cell_centres(cfg)
    blob = (np.abs(X - 0.4) < 0.15) & (np.abs(Y - 0.55) < 0.2)
    f["rho"] = np.where(blob, 4.0, 1.0)
    f["p"] = np.where(blob, 10.0, 1.0)
    g = pond.Context(cfg, f, precision=precision)
    g.set_iter_split(1)
    U0 = g.conserved().sum(axis=1)
    st = g.step(30)
    U1 = g.conserved().sum(axis=1)
    scale = np.abs(g.conserved()).sum(axis=1)
    assert st["tail_faces"] > 100
    assert np.all(np.abs(U1 - U0) <= 1e-13 * scale)


@pytest.mark.parametrize("layout", ["hermite", "populations"])
def test_2d_tiles_bitwise_identical(orc, layout):
    """Every 2D tile shape gives bitwise-identical FP64 results (the LDS halo is complete),
    with the state held as coefficients or as populations; the tiles cover every LDS plane
    stride of the FP64 face kernel (256: 8 x 8, 32 x 2; 384: 16 x 16; 512: 32 x 8, 64 x 4)."""
    from paper_2203_05477_amd import pond

    cfg, f = W.double_mach(70, 30)
    outs = []
    for bx, by in ((8, 8), (16, 16), (32, 2), (64, 4), (32, 8)):
        g = pond.Context(cfg, f, precision="fp64")
        if layout == "populations":
            g.set_state_layout("populations")
        g.set_tiles(bx, by, 256)
        g.step(12)
        outs.append((g.conserved(), g.face_frames()))
    for U, F in outs[1:]:
        assert np.array_equal(U, outs[0][0]) and np.array_equal(F, outs[0][1])


def _face_cells(cfg, faces):
    """Cells (row, column) on either side of the given face indices (x-faces first)."""
    nx, ny = cfg["nx"], cfg["ny"]
    nfx = (nx + 1) * ny
    cells = set()
    for k in faces:
        if k < nfx:
            i, j = k % (nx + 1), k // (nx + 1)
            cells.update({(j, i - 1), (j, i)})
        else:
            i, j = (k - nfx) % nx, (k - nfx) // nx
            cells.update({(j - 1, i), (j, i)})
    return cells


def _lockstep(orc, cfg, f, steps):
    """Step the GPU path and the oracle side by side. While every face ends its iteration
    the same way on both sides (converged, or not converged and replaced by the fallback
    state), the conserved fields agree to TOL64. A face whose iteration sits at the
    max_iter cut can end differently under different rounding orders (both outcomes are
    results of the method); at the first such step the fields may differ only in the cells
    next to those faces, and the comparison ends there. Returns the number of steps
    compared element by element."""
    g, o = _pair(orc, cfg, f)
    nx, ny = cfg["nx"], cfg["ny"]
    for k in range(steps):
        o.step()
        g.step(1)
        assert g.time()[0] == pytest.approx(o.t, rel=1e-14)
        e = _relerr(g.conserved(), o.conserved())
        split = np.nonzero((g.face_iters() > 0) != (o.face_iters() > 0))[0]
        if len(split) == 0:
            assert e.max() <= TOL64, (k, e)
            continue
        Ug, Uo = g.conserved(), o.conserved()
        scale = np.abs(Uo).max(axis=1, keepdims=True)
        d = (np.abs(Ug - Uo) / scale).max(axis=0).reshape(ny, nx)
        off = {tuple(c) for c in np.argwhere(d > TOL64)}
        assert off <= _face_cells(cfg, split), (k, sorted(off - _face_cells(cfg, split))[:5])
        _print("decisions split", step=k, faces=len(split), cells=len(off))
        return k
    return steps


@pytest.mark.parametrize("speed,steps,min_steps", [(1.0, 6, 2), (30.0, 12, 1)])
def test_jet_small_fp64(orc, speed, steps, min_steps):
    """The jet set-up on 64 x 64 cells at jet speed 1 and at the paper's 30 (Mach 80):
    fixed inflow window, the boundary states in the time step, strong shear at the inflow
    and faces that reach the iteration cap."""
    cfg, f = W.jet(64, 64, tol=1e-13, speed=speed)
    _print("case", name="jet", nx=64, ny=64, speed=speed)
    n = _lockstep(orc, cfg, f, steps)
    _print("jet", speed=speed, lockstep_steps=n)
    assert n >= min_steps


def test_shocked_interface_small_fp64(orc):
    """The shocked heavy/light interface on 128 x 32 cells (periodic in y), 25 steps."""
    cfg, f = W.shocked_interface(128, 32, tol=1e-13)
    _print("case", name="shocked_interface", nx=128, ny=32)
    g, o = _pair(orc, cfg, f)
    for _ in range(25):
        o.step()
        g.step(1)
    e = _relerr(g.conserved(), o.conserved())
    _print("shocked_interface", err=e.max())
    assert e.max() <= TOL64


def test_launch_shapes_above_256_threads_are_rejected():
    """Every kernel is compiled for at most 256 threads per block: larger shapes are
    refused when they are set, not when a launch fails."""
    from paper_2203_05477_amd import pond

    cfg, f = W.double_mach(64, 16)
    g = pond.Context(cfg, f, precision="fp64")
    for bx, by, cb in ((32, 16, 256), (16, 8, 512), (8, 4, 256)):
        with pytest.raises(pond.PondError):
            g.set_tiles(bx, by, cb)
    g.set_tiles(16, 16, 256)
    g.step(2)
    cfg, f = W.shock_tube(64)
    h = pond.Context(cfg, f, precision="fp64")
    with pytest.raises(pond.PondError):
        h.set_tiles(512, 1, 256)
    h.set_tiles(192, 1, 128)
    h.step(2)
