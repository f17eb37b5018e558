"""The further 1D Riemann problems the paper prints (Lax, Sec. IV.A.2; strong shock tube,
double rarefaction and Le Blanc, Sec. IV.B; the 1D jet, Sec. IV.C.5) on the oracle, pinned
to the exact Riemann solution and to conservation with the exact boundary fluxes."""
import numpy as np
import pytest

import exact_riemann as ER
from paper_2203_05477_amd import workloads as W

CASES = ("lax", "strong_shock", "le_blanc", "jet_1d")


def _run(orc, name, nx, stop_on_invalid=True):
    cfg, f = W.riemann_case(name, nx=nx, tol=1e-10)
    s = orc.Sim(cfg, f["rho"], f["ux"], f.get("uy"), f["p"])
    t_end = cfg["t_end"]
    steps = 0
    while s.t < t_end * (1 - 1e-12):
        s.step(t_end)
        steps += 1
        if stop_on_invalid:
            r, _, _, T = s.fields()
            assert r.min() > 0 and T.min() > 0, (name, nx, steps)
    return cfg, s, steps


def _l1(cfg, s):
    left, right, xi, (a, b), g = W.RIEMANN_CASES[cfg["name"]][:5]
    ex = ER.cell_average(left, right, g, np.linspace(a, b, cfg["nx"] + 1), xi, s.t)
    U = s.conserved()
    return np.array([np.abs(U[k] - ex[k]).sum() / np.abs(ex[k]).sum() for k in range(3)])


# relative L1 error of (rho, rho u, rho E) at 400 cells: the oracle's values are
# 9.9e-3 / 4.7e-2 / 5.0e-3 / 2.7e-2 in density; the bounds leave about 20% room
L1_400 = {"lax": (0.012, 0.017, 0.003), "strong_shock": (0.057, 0.091, 0.013),
          "le_blanc": (0.006, 0.022, 0.011), "jet_1d": (0.032, 0.027, 0.021)}


@pytest.mark.parametrize("name", CASES)
def test_printed_riemann_problem_converges_to_exact_solution(orc, name):
    """Every conserved field's relative L1 error against the exact solution falls at each
    doubling 100 -> 200 -> 400 cells and is small at 400 cells; the final time is met
    exactly (last step clipped)."""
    errs = []
    for nx in (100, 200, 400):
        cfg, s, steps = _run(orc, name, nx)
        assert s.t == pytest.approx(cfg["t_end"], rel=1e-14)
        errs.append(_l1(cfg, s))
    e100, e200, e400 = errs
    print(name, e100, e200, e400)
    assert np.all(e200 < e100) and np.all(e400 < e200)
    assert np.all(e400 < L1_400[name])


def _euler_flux(state, gamma):
    r, u, p = state
    E = p / (gamma - 1.0) + 0.5 * r * u * u
    return np.array([r * u, r * u * u + p, u * (E + p)])


@pytest.mark.parametrize("name", CASES)
def test_conservation_with_exact_boundary_fluxes(orc, name):
    """Until a wave reaches an end of the tube, both outflow boundary faces see a uniform
    equilibrium state, whose face state is that equilibrium itself, so the flux through
    them is the Euler flux of the initial states; the interior fluxes telescope. Hence
    sum_j U_j dx = sum_j U_j(0) dx + t (F(left) - F(right)) up to round-off."""
    cfg, f = W.riemann_case(name, nx=200, tol=1e-10)
    left, right, xi, (a, b), g, t_end = W.RIEMANN_CASES[name][:6]
    # no wave of the exact solution reaches either end before t_end
    ex = ER.cell_average(left, right, g, np.linspace(a, b, 201), xi, t_end)
    assert ex[0][0] == pytest.approx(left[0], rel=1e-12)
    assert ex[0][-1] == pytest.approx(right[0], rel=1e-12)
    s = orc.Sim(cfg, f["rho"], f["ux"], None, f["p"])
    U0 = s.conserved().sum(axis=1)
    while s.t < t_end * (1 - 1e-12):
        s.step(t_end)
    U1 = s.conserved().sum(axis=1)
    dx = (b - a) / 200
    pred = U0 + s.t / dx * (_euler_flux(left, g) - _euler_flux(right, g))
    scale = np.maximum(np.abs(pred), np.abs(U0))
    assert np.all(np.abs(U1 - pred) <= 1e-11 * scale), (U1 - pred) / scale


def test_double_rarefaction_symmetric_up_to_known_departure(orc):
    """KNOWN DEPARTURE from Sec. IV.B: the paper reports the printed double rarefaction
    (p = 0.1 on both sides, u = -2 | 2) in good agreement with the exact solution at
    t = 0.1 on 800 cells; under the readings adopted here the step cannot hold it (every
    reading tried is listed in the design notes with its failing step). This test pins how
    the case departs, not what the paper shows: the exact solution opens a true vacuum
    (2 (c_L + c_R)/(gamma - 1) < u_R - u_L); the step keeps the mirror symmetry exactly
    (rho even, u odd) while the two centre cells drain, and the internal energy next to the
    centre turns negative within ten steps with the Van Leer limiter and within a hundred
    with minmod. The paper's outcome is asserted, as an expected failure, by
    test_double_rarefaction_reaches_the_printed_time."""
    left, right, _, _, g = W.RIEMANN_CASES["double_rarefaction"][:5]
    cl, cr = (np.sqrt(g * s[2] / s[0]) for s in (left, right))
    assert 2.0 * (cl + cr) / (g - 1.0) < right[1] - left[1]
    for nx in (100, 800):
        for lim in ("vanleer", "minmod"):
            cfg, f = W.riemann_case("double_rarefaction", nx=nx, tol=1e-10)
            cfg["limiter"] = lim
            s = orc.Sim(cfg, f["rho"], f["ux"], None, f["p"])
            failed = None
            for n in range(1, 101):
                s.step(cfg["t_end"])
                r, u, _, T = s.fields()
                if not (T.min() > 0):
                    failed = n
                    break
                assert np.abs(r - r[::-1]).max() <= 1e-12
                assert np.abs(u + u[::-1]).max() <= 1e-12
            k = int(np.argmin(T))
            print("double rarefaction", nx, lim, "T <= 0 at step", failed, "cell", k)
            assert failed is not None and (lim == "minmod" or failed <= 10)
            assert abs(k + 0.5 - nx / 2) <= 4


@pytest.mark.xfail(strict=True, reason="known departure from Sec. IV.B: the double rarefaction "
                   "loses positivity next to the centre under every reading tried")
def test_double_rarefaction_reaches_the_printed_time(orc):
    """The paper's outcome (Sec. IV.B): the run reaches t = 0.1 on 200 cells with positive
    density and temperature everywhere, and its density is within 10% (relative L1) of the
    exact solution. Expected to fail under the readings adopted here."""
    from exact_riemann import sample

    cfg, f = W.riemann_case("double_rarefaction", nx=200, tol=1e-10)
    s = orc.Sim(cfg, f["rho"], f["ux"], None, f["p"])
    while s.t < cfg["t_end"] * (1 - 1e-12):
        s.step(cfg["t_end"])
        r, _, _, T = s.fields()
        assert r.min() > 0 and T.min() > 0, f"T <= 0 at step {s.steps}"
    left, right, xi, _, g = W.RIEMANN_CASES["double_rarefaction"][:5]
    x = (np.arange(cfg["nx"]) + 0.5) / cfg["nx"]
    rex = sample(left, right, g, (x - xi) / s.t)[0]
    assert np.abs(r - rex).sum() <= 0.1 * np.abs(rex).sum()


def test_blast_waves_closed_tube_invariants(orc):
    """Two interacting blast waves (Sec. IV.B) between reflecting ends: mass and energy of
    the closed tube are kept through the whole run to t = 0.038, and the collision of the
    two waves compresses the gas well above the 4x of a single strong shock at gamma 1.4
    (the peak of this problem's known solution is near 6).

    The bar is 1e-12 relative, not the 1e-13 of the smooth cases: each cell projects the
    moments of its faces into its own frame before summing the flux, so the two cells of a
    face add its flux through two different projections. Across the blast fronts the
    temperatures of face and cell differ by up to 1e5 (1000 against 0.01), and the rounding
    of those projections no longer cancels: the totals drift by about 1.6e-14 (mass) per
    step, 2e-13 (mass) and 6e-13 (energy) relative over the 5,300 steps."""
    cfg, f = W.blast_waves(400)
    s = orc.Sim(cfg, f["rho"], f["ux"], None, f["p"])
    U0 = s.conserved().sum(axis=1)
    while s.t < cfg["t_end"] * (1 - 1e-12):
        s.step(cfg["t_end"])
    U1 = s.conserved().sum(axis=1)
    assert abs(U1[0] - U0[0]) <= 1e-12 * U0[0] and abs(U1[2] - U0[2]) <= 1e-12 * U0[2]
    r, _, _, T = s.fields()
    assert T.min() > 0 and 4.5 < r.max() < 6.5
