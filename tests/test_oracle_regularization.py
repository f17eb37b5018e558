"""Pins of the oracle's alternative regularization (Sec. II.C: the moments of order 0..3
keep their values, the remaining Q - q moments are set to equilibrium in the new frame,
and the populations follow by moment inversion), and of whole steps that use it."""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W


def _rand_state(rng, orc, dim=2):
    c, Wt = orc.lattice(dim)
    f = Wt * (1.0 + 0.4 * rng.uniform(-1, 1, Wt.size)) * rng.uniform(0.2, 5.0)
    u = rng.uniform(-3, 3, dim)
    T = rng.uniform(0.1, 4.0)
    return f, u, T


def _gauss_weights_1d(orc, d):
    """Weights on the four D1Q4 nodes whose first four moments are those of a unit-variance
    Gaussian centred at d (1, d, d^2 + 1, d^3 + 3 d): the 1D factor of the product-form
    equilibrium, from a 4 x 4 Vandermonde solve."""
    c = orc.lattice(1)[0].ravel()
    V = np.vstack([c ** k for k in range(4)])
    return np.linalg.solve(V, np.array([1.0, d, d * d + 1.0, d ** 3 + 3.0 * d]))


def _kappa(u, T):
    """Conditioning of the passage between lab moments up to degree 3 and frame-relative
    ones: their binomial expansion sums terms up to (|u|/sqrt T)^3 times the result."""
    return (1.0 + np.abs(u).max() / np.sqrt(T)) ** 3


def test_product_form_equilibrium_is_reproduced_exactly(orc):
    """A product-form equilibrium of the new frame's lattice (density rho, velocity u,
    the frame's temperature) has all 16 moments at the values the construction sets, so
    the transformation must return it population by population; the Grad projection,
    whose fast moments follow the Grad closure instead, does not."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        rho = rng.uniform(0.1, 10)
        u1, T1 = rng.uniform(-3, 3, 2), rng.uniform(0.1, 4)
        u = u1 + rng.uniform(-1.0, 1.0, 2) * np.sqrt(T1)
        d = (u - u1) / np.sqrt(T1)
        wx, wy = _gauss_weights_1d(orc, d[0]), _gauss_weights_1d(orc, d[1])
        f = rho * np.array([wx[i % 4] * wy[i // 4] for i in range(16)])
        M = orc.moments(2, 3, f, u1, T1)
        g = orc.eq_project(2, M, u1, T1)
        assert np.abs(g - f).max() <= 1e-13 * _kappa(u1, T1) * np.abs(f).max()
        gg = orc.grad_project(2, 3, M, u1, T1)
        assert np.abs(gg - f).max() > 1e-6 * np.abs(f).max() or np.abs(d).max() < 1e-3


def test_slow_moments_are_kept(orc):
    """M_0..M_3 of the result in the new frame equal those of the input (any frames), to
    round-off times the conditioning of the lab/frame-relative passage."""
    rng = np.random.default_rng(12)
    for _ in range(30):
        f, u0, T0 = _rand_state(rng, orc)
        M = orc.moments(2, 3, f, u0, T0)
        u1, T1 = rng.uniform(-3, 3, 2), rng.uniform(0.1, 4)
        g = orc.eq_project(2, M, u1, T1)
        M1 = orc.moments(2, 3, g, u1, T1)
        assert np.abs(M1 - M).max() <= 1e-13 * _kappa(u1, T1) * np.abs(M).max()


def test_galilean_invariance(orc):
    """Shifting the state and the target frame by one lab velocity U leaves the populations
    unchanged (they live on the frame-relative lattice). A construction on lab-velocity
    monomials would fail this: its fast moments mix in powers of the frame's own lab
    velocity."""
    rng = np.random.default_rng(13)
    for _ in range(20):
        f, u0, T0 = _rand_state(rng, orc)
        u1, T1 = u0 + rng.uniform(-1, 1, 2), T0 * rng.uniform(0.5, 2)
        U = rng.uniform(-5, 5, 2)
        g = orc.eq_project(2, orc.moments(2, 3, f, u0, T0), u1, T1)
        gU = orc.eq_project(2, orc.moments(2, 3, f, u0 + U, T0), u1 + U, T1)
        assert np.abs(gU - g).max() <= 1e-13 * _kappa(u1 + U, T1) * np.abs(g).max()


def test_idempotent_and_comoving_equilibrium(orc):
    """Transforming a result again into the same frame returns it; the co-moving
    equilibrium rho W_i is kept in its own frame."""
    rng = np.random.default_rng(14)
    _, Wt = orc.lattice(2)
    for _ in range(20):
        f, u0, T0 = _rand_state(rng, orc)
        u1, T1 = rng.uniform(-3, 3, 2), rng.uniform(0.1, 4)
        g = orc.eq_project(2, orc.moments(2, 3, f, u0, T0), u1, T1)
        g2 = orc.eq_project(2, orc.moments(2, 3, g, u1, T1), u1, T1)
        assert np.abs(g2 - g).max() <= 1e-13 * _kappa(u1, T1) * np.abs(g).max()
        rho = rng.uniform(0.1, 10)
        e = orc.eq_project(2, orc.moments(2, 3, rho * Wt, u1, T1), u1, T1)
        assert np.abs(e - rho * Wt).max() <= 1e-13 * _kappa(u1, T1) * rho


def test_one_dimension_has_no_fast_moments(orc):
    """D1Q4 carries exactly M_0..M_3: the transformation is the Grad projection."""
    rng = np.random.default_rng(15)
    for _ in range(20):
        f, u0, T0 = _rand_state(rng, orc, dim=1)
        M = orc.moments(1, 3, f, u0, T0)
        u1, T1 = rng.uniform(-3, 3, 1), rng.uniform(0.1, 4)
        assert np.array_equal(orc.eq_project(1, M, u1, T1), orc.grad_project(1, 3, M, u1, T1))


def _sim(orc, cfg, f):
    return orc.Sim(cfg, f["rho"], f["ux"], f.get("uy"), f["p"])


def test_step_conserves_and_keeps_uniform_flow(orc):
    """Whole steps with the alternative regularization: the totals of a periodic box are
    conserved to round-off (the flux form telescopes whatever the face populations), a
    uniform flow stays uniform from any seed, and the result differs from the Grad
    projection's once the flow is not uniform."""
    cfg, f = W.random_smooth(2, 12, 10, seed=5, cfl=0.3, tol=1e-13)
    cfg["regularization"] = "eq"
    s = _sim(orc, cfg, f)
    U0 = s.conserved().sum(axis=1)
    for _ in range(5):
        s.step()
    U1 = s.conserved().sum(axis=1)
    assert np.all(np.abs(U1 - U0) <= 1e-13 * np.abs(U0).max())
    g = dict(cfg, regularization="grad")
    sg = _sim(orc, g, f)
    for _ in range(5):
        sg.step()
    assert np.abs(sg.conserved() - s.conserved()).max() > 1e-10
    cfg, f = W.uniform(2, 6, 5, rho=1.3, u=(0.7, -0.4), p=0.9, tol=1e-13)
    cfg["regularization"] = "eq"
    s = _sim(orc, cfg, f)
    for _ in range(3):
        s.step()
    r, ux, uy, T = s.fields()
    assert np.abs(r - 1.3).max() < 1e-13 and np.abs(ux - 0.7).max() < 1e-13
    assert np.abs(uy + 0.4).max() < 1e-13 and np.abs(T - 0.9 / 1.3).max() < 1e-13


def test_step_one_dimension_is_unchanged(orc):
    """In 1D the two regularizations are the same transformation: the same bits."""
    cfg, f = W.shock_tube(60)
    a = _sim(orc, cfg, f)
    b = _sim(orc, dict(cfg, regularization="eq"), f)
    for _ in range(20):
        a.step()
        b.step()
    assert np.array_equal(a.conserved(), b.conserved())


def test_step_transpose_equivariance(orc):
    """Swapping x and y in the initial state swaps them in the result (the construction
    treats both axes alike)."""
    cfg, f = W.random_smooth(2, 8, 8, seed=9, cfl=0.3, tol=1e-13)
    cfg["regularization"] = "eq"
    tr = lambda a: a.reshape(8, 8).T.ravel()
    s = _sim(orc, cfg, f)
    ft = {"rho": tr(f["rho"]), "ux": tr(f["uy"]), "uy": tr(f["ux"]), "p": tr(f["p"])}
    st = _sim(orc, cfg, ft)
    for _ in range(3):
        s.step()
        st.step()
    r, ux, uy, T = s.fields()
    rt, uxt, uyt, Tt = st.fields()
    assert np.abs(tr(r) - rt).max() < 1e-12
    assert np.abs(tr(ux) - uyt).max() < 1e-12
    assert np.abs(tr(T) - Tt).max() < 1e-12
