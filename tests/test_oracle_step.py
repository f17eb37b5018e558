"""Pins of the oracle's whole finite-volume step (Sec. III.B) against invariants,
closed forms, exact Riemann solutions and the paper's printed set-up values."""
import math

import numpy as np
import pytest

import exact_riemann as ER
from conftest import read_golden
from paper_2203_05477_amd import workloads as W


def _sim(orc, cfg, f):
    return orc.Sim(cfg, f["rho"], f["ux"], f.get("uy"), f["p"])


@pytest.mark.parametrize("dim", [1, 2])
def test_uniform_flow_stays_uniform_any_seed(orc, dim):
    """A uniform state is a fixed point of the step whatever the face seeds are: every
    stencil cell is equal, slopes vanish, and any frame reproduces the exact moments."""
    cfg, f = W.uniform(dim, 12, 8 if dim == 2 else 1, tol=1e-13)
    s = _sim(orc, cfg, f)
    s.step()
    rng = np.random.default_rng(0)
    fr = s.face_frames()
    fr[:, :dim] += rng.uniform(-0.5, 0.5, (fr.shape[0], dim))
    fr[:, dim] *= rng.uniform(0.5, 2.0, fr.shape[0])
    s.set_face_frames(fr)
    for _ in range(3):
        s.step()
    r, ux, uy, T = s.fields()
    assert np.abs(r - 1.0).max() < 1e-13
    assert np.abs(ux - 0.3).max() < 1e-13
    assert np.abs(T - 0.7).max() < 1e-13
    if dim == 2:
        assert np.abs(uy + 0.2).max() < 1e-13


@pytest.mark.parametrize("dim,nx,ny", [(1, 64, 1), (2, 24, 16)])
def test_periodic_conservation(orc, dim, nx, ny):
    """The FV update is conservative (Sec. III.B): on a periodic domain the totals of
    rho, rho u and rho E stay constant to round-off."""
    cfg, f = W.random_smooth(dim, nx, ny, seed=3, cfl=0.3, tol=1e-12)
    s = _sim(orc, cfg, f)
    U0 = s.conserved().sum(axis=1)
    for _ in range(10):
        s.step()
    U1 = s.conserved().sum(axis=1)
    scale = np.abs(s.conserved()).sum(axis=1)
    assert np.all(np.abs(U1 - U0) <= 1e-13 * scale)
    # a dropped flux term or a wrong sign would change the totals
    assert s.steps == 10


def test_closed_reflecting_box_conserves_mass(orc):
    """Reflecting walls on all sides (Sec. IV.C.2 set-up type): mass and energy exact."""
    cfg = W.base_config(2, 20, 20, bc=("reflect",) * 4, tol=1e-12)
    X, Y = W.cell_centres(cfg)
    inside = (X - 0.4) ** 2 + (Y - 0.4) ** 2 < 0.3 ** 2
    f = {"rho": np.where(inside, 5.0, 1.0), "ux": np.zeros(X.size), "uy": np.zeros(X.size),
         "p": np.where(inside, 5.0, 1.0)}
    s = _sim(orc, cfg, f)
    U0 = s.conserved().sum(axis=1)
    for _ in range(8):
        s.step()
    U1 = s.conserved().sum(axis=1)
    assert abs(U1[0] - U0[0]) <= 1e-13 * U0[0]
    assert abs(U1[3] - U0[3]) <= 1e-13 * U0[3]


def _l1_vs_exact(orc, nx):
    cfg, f = W.shock_tube(nx, tol=1e-10)
    s = _sim(orc, cfg, f)
    while s.t < 0.2 * (1 - 1e-12):
        s.step(0.2)
    U = s.conserved()
    ex = ER.cell_average((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, np.linspace(0, 1, nx + 1),
                         0.5, 0.2)
    return np.array([np.abs(U[k] - ex[k]).sum() / np.abs(ex[k]).sum() for k in range(3)]), s


def test_shock_tube_converges_to_exact_solution(orc):
    """The 400-cell shock tube (Sec. IV.A.1 type) against the exact Riemann solution:
    small relative L1 error, decreasing under refinement."""
    e100, _ = _l1_vs_exact(orc, 100)
    e200, _ = _l1_vs_exact(orc, 200)
    e400, s = _l1_vs_exact(orc, 400)
    assert np.all(e400 < [0.03, 0.08, 0.03])
    assert np.all(e200 < e100) and np.all(e400 < e200)
    assert s.t == pytest.approx(0.2, abs=1e-14)


def test_smooth_wave_second_order(orc):
    """A density wave advected in a uniform-pressure flow (periodic): the MUSCL
    reconstruction at the half-step departure point gives about second order (a dropped
    slope or a full-step departure point gives first order)."""
    errs = []
    for nx in (32, 64, 128):
        cfg = W.base_config(1, nx, cfl=0.3, mu=1e-6, tol=1e-12, bc=("periodic",) * 4)
        x, _ = W.cell_centres(cfg)
        dx = 1.0 / nx
        # cell averages of 1 + 0.2 sin(2 pi x)
        rho = 1.0 + 0.2 * (np.cos(2 * np.pi * (x - dx / 2)) - np.cos(2 * np.pi * (x + dx / 2))) / (2 * np.pi * dx)
        s = orc.Sim(cfg, rho, np.full(nx, 1.0), None, np.full(nx, 1.0))
        tend = 0.25
        while s.t < tend * (1 - 1e-12):
            s.step(tend)
        r, _, _, _ = s.fields()
        ex = 1.0 + 0.2 * (np.cos(2 * np.pi * (x - dx / 2 - tend)) - np.cos(2 * np.pi * (x + dx / 2 - tend))) / (2 * np.pi * dx)
        errs.append(np.abs(r - ex).mean())
    order = math.log2(errs[1] / errs[2])
    assert order > 1.4, errs


def test_transpose_equivariance(orc):
    """Swapping x and y (fields, velocities, boundaries) transposes the solution."""
    cfg, f = W.random_smooth(2, 12, 9, seed=4, tol=1e-13, bc="outflow")
    s = _sim(orc, cfg, f)
    cfgT = dict(cfg)
    cfgT["nx"], cfgT["ny"] = cfg["ny"], cfg["nx"]
    cfgT["x0"], cfgT["x1"], cfgT["y0"], cfgT["y1"] = cfg["y0"], cfg["y1"], cfg["x0"], cfg["x1"]
    tr = lambda a: a.reshape(cfg["ny"], cfg["nx"]).T.ravel()
    sT = orc.Sim(cfgT, tr(f["rho"]), tr(f["uy"]), tr(f["ux"]), tr(f["p"]))
    for _ in range(4):
        s.step()
        sT.step()
    r, ux, uy, T = s.fields()
    rT, uxT, uyT, TT = sT.fields()
    assert np.abs(tr(r) - rT).max() < 1e-12
    assert np.abs(tr(ux) - uyT).max() < 1e-12
    assert np.abs(tr(uy) - uxT).max() < 1e-12
    assert np.abs(tr(T) - TT).max() < 1e-12


def test_mirror_symmetry(orc):
    """A state symmetric under x -> -x stays symmetric (u_x odd, rest even)."""
    cfg = W.base_config(2, 16, 6, x0=-1.0, x1=1.0, tol=1e-13, bc=("reflect",) * 4)
    X, Y = W.cell_centres(cfg)
    rho = 1.0 + 0.5 * np.exp(-8 * X ** 2) + 0.1 * Y
    ux = 0.3 * np.sin(np.pi * X)
    f = {"rho": rho, "ux": ux, "uy": 0.1 * np.cos(np.pi * X), "p": 1.0 + 0.2 * np.exp(-8 * X ** 2)}
    s = _sim(orc, cfg, f)
    for _ in range(4):
        s.step()
    r, ux, uy, T = s.fields()
    m = lambda a: a.reshape(6, 16)[:, ::-1].ravel()
    assert np.abs(r - m(r)).max() < 1e-12
    assert np.abs(ux + m(ux)).max() < 1e-12
    assert np.abs(T - m(T)).max() < 1e-12


def test_y_uniform_2d_stays_y_uniform(orc):
    cfg, f = W.riemann_1d((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), nx=40)
    cfg2 = W.base_config(2, 40, 6, tol=1e-13, bc=("outflow", "outflow", "periodic", "periodic"))
    s = orc.Sim(cfg2, np.tile(f["rho"], 6), np.tile(f["ux"], 6), np.zeros(240), np.tile(f["p"], 6))
    for _ in range(6):
        s.step()
    r, ux, uy, T = s.fields()
    R = r.reshape(6, 40)
    assert np.abs(R - R[0]).max() < 1e-13
    assert np.abs(uy).max() < 1e-13


def test_dmr_post_shock_state_matches_paper():
    """The normal-shock relations used to build the Mach-10 set-up reproduce the printed
    post-shock state (Sec. IV.C.4)."""
    g = read_golden()
    cfg, _ = W.double_mach(24, 6)
    post = [eval(t.replace("sqrt3", "math.sqrt(3)"), {"math": math}) for t in g["dmr_post"]]
    pre = [float(t) for t in g["dmr_pre"]]
    assert cfg["pre"] == pytest.approx(pre)
    assert cfg["post"] == pytest.approx(post, rel=1e-12, abs=1e-12)


def test_jet_and_strong_shock_numbers():
    """Mach 80 of the jet (Sec. IV.C.5) and the 1e5 temperature ratio of the strong shock
    tube (Sec. IV.B.1) follow from the printed states."""
    g = read_golden()
    rho, u, p = (float(t) for t in g["jet_state"])
    mach = u / math.sqrt(5.0 / 3.0 * p / rho)
    assert abs(mach - float(g["jet_mach"][0])) < 1.5
    rl, _, pl = (float(t) for t in g["strong_shock_left"])
    rr, _, pr = (float(t) for t in g["strong_shock_right"])
    assert (pl / rl) / (pr / rr) == pytest.approx(float(g["strong_shock_T_ratio"][0]))


def test_exact_riemann_solver_relations():
    """The test reference itself: p* solves the pressure equation, the shock satisfies the
    Rankine-Hugoniot jump conditions and the rarefaction keeps p/rho^gamma."""
    left, right, g = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4
    ps, us = ER.star_state(left, right, g)
    assert abs(ER.residual(left, right, g, ps)) < 1e-14
    xi = np.linspace(-2, 2, 4001)
    r, u, p = ER.sample(left, right, g, xi)
    # right shock: states just behind and ahead
    k = np.where(np.abs(np.diff(r)) > 0.05)[0][-1]
    rs, uss, pss = r[k - 1], u[k - 1], p[k - 1]
    S = (rs * uss - right[0] * right[1]) / (rs - right[0])
    assert rs * (uss - S) == pytest.approx(right[0] * (right[1] - S), rel=1e-9)
    mom = lambda rr, uu, pp: rr * (uu - S) * uu + pp
    assert mom(rs, uss, pss) == pytest.approx(mom(*right), rel=1e-9)
    # rarefaction: isentropic
    fan = (xi > -1.1) & (xi < 0.0) & (np.abs(u) > 1e-3) & (u < us - 1e-3)
    assert np.allclose(p[fan] / r[fan] ** g, left[2] / left[0] ** g, rtol=1e-10)


def test_time_step_includes_the_prescribed_boundary_states(orc):
    """CFL = max over every population that crosses a face of |v_a| dt / dx_a (Sec. IV):
    at t = 0 the jet's interior is ambient gas at rest, and the fastest populations are
    those the fixed jet inflow sends through the left boundary, so
    dt = CFL dx / (30 + sqrt(T_jet) c_max) with c_max = sqrt(3 + sqrt 6)."""
    cfg, f = W.jet(32, 32, tol=1e-10)
    s = _sim(orc, cfg, f)
    s.step()
    cmax = math.sqrt(3.0 + math.sqrt(6.0))
    dx = 1.0 / 32
    assert s.last["dt"] == pytest.approx(0.2 * dx / (30.0 + math.sqrt(0.4127 / 5.0) * cmax), rel=1e-14)
    # a closed periodic box has no boundary states: dt follows the interior alone
    cfg, f = W.uniform(2, 8, 8, rho=1.0, u=(0.3, -0.2), p=0.7, tol=1e-13)
    s = _sim(orc, cfg, f)
    s.step()
    assert s.last["dt"] == pytest.approx(0.2 / 8 / (0.3 + math.sqrt(0.7) * cmax), rel=1e-14)


def test_explosion_box_setup_and_invariants(orc):
    """Explosion in a box (Sec. IV.C.2): the set-up takes the printed states, and in the
    closed reflecting box mass and energy are exact while the state keeps its symmetry
    about the diagonal x = y (the circle is centred on it)."""
    g = read_golden()
    cfg, f = W.explosion_box(32)
    inside = [float(t) for t in g["explosion_box_inside"]]
    outside = [float(t) for t in g["explosion_box_outside"]]
    k_in, k_out = int(np.argmax(f["rho"])), int(np.argmin(f["rho"]))
    assert [f[q][k_in] for q in ("rho", "ux", "uy", "p")] == inside
    assert [f[q][k_out] for q in ("rho", "ux", "uy", "p")] == outside
    s = _sim(orc, cfg, f)
    U0 = s.conserved().sum(axis=1)
    for _ in range(20):
        s.step()
    U1 = s.conserved().sum(axis=1)
    assert abs(U1[0] - U0[0]) <= 1e-13 * U0[0] and abs(U1[3] - U0[3]) <= 1e-13 * U0[3]
    r, ux, uy, _ = s.fields()
    tr = lambda a: a.reshape(32, 32).T.ravel()
    assert np.abs(tr(r) - r).max() < 1e-12 and np.abs(tr(ux) - uy).max() < 1e-12


@pytest.mark.xfail(strict=True, reason="known departure from Sec. IV.C.5: the Mach-80 jet loses "
                   "positivity at the jet edge next to the inflow under every reading tried")
def test_jet_on_the_paper_domain_keeps_running(orc):
    """The paper's 2D jet (Sec. IV.C.5) on its own domain [0,2] x [-0.5,0.5], here on a
    100 x 50 grid: the run keeps positive density and temperature for 300 steps while the
    bow shock moves into the ambient gas. Expected to fail under the readings adopted here (the
    shear layer where the jet edge meets the fixed inflow boundary reaches T <= 0 within
    about 50 steps at this resolution)."""
    cfg, f = W.jet(100, 50, x1=2.0, tol=1e-10)
    s = _sim(orc, cfg, f)
    for k in range(300):
        s.step()
        r, _, _, T = s.fields()
        assert r.min() > 0 and T.min() > 0, f"T <= 0 at step {k + 1}"
