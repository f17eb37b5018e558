"""Pins of the oracle's building blocks against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: printed values
(Table I), closed-form quadrature identities, the defining moment-invariance
condition of the Grad projection (Sec. II.C), a library linear solve for the 1D
special case, and the definitions of the DUGKS variable transforms (Sec. III.B).
"""
import math

import numpy as np
import pytest

from conftest import read_golden

S6 = math.sqrt(6.0)


def _val(tok):
    return float(eval(tok.replace("sqrt6", "math.sqrt(6)").replace("sqrt3", "math.sqrt(3)"),
                      {"math": math}))


def test_table1_nodes_and_weights(orc):
    """Table I: D1Q4 nodes +-sqrt(3 -+ sqrt 6), weights (3 +- sqrt 6)/12."""
    g = read_golden()
    c, W = orc.lattice(1)
    c = c[:, 0]
    n2 = sorted(_val(t) for t in g["d1q4_nodes_squared"])
    assert np.allclose(sorted(set(np.round(c * c, 14))), n2, rtol=0, atol=1e-14)
    w_inner, w_outer = (_val(t) for t in g["d1q4_weights"])
    for ci, wi in zip(c, W):
        expect = w_inner if abs(ci * ci - n2[0]) < 1e-12 else w_outer
        assert wi == pytest.approx(expect, abs=1e-15)
    # D2Q16 weights are products (Sec. II.A), and so are those of its 3D analogue D3Q64
    c2, W2 = orc.lattice(2)
    for i in range(16):
        assert W2[i] == pytest.approx(W[i % 4] * W[i // 4], abs=1e-16)
        assert c2[i, 0] == c[i % 4] and c2[i, 1] == c[i // 4]
    c3, W3 = orc.lattice(3)
    assert len(W3) == 64
    for i in range(64):
        ix, iy, iz = i % 4, (i // 4) % 4, i // 16
        assert W3[i] == pytest.approx(W[ix] * W[iy] * W[iz], abs=1e-16)
        assert (c3[i, 0], c3[i, 1], c3[i, 2]) == (c[ix], c[iy], c[iz])


def test_d3q64_mixed_moments_are_normal_moments(orc):
    """D3Q64 integrates every monomial c_x^a c_y^b c_z^c with a, b, c <= 7 like the standard
    normal distribution in 3D (product of 1D moments, numpy's probabilists' Gauss-Hermite
    rule as the independent reference); a degree-8 power along one axis is not exact."""
    c, W = orc.lattice(3)
    x, w = np.polynomial.hermite_e.hermegauss(4)
    w = w / w.sum()
    normal = [1, 0, 1, 0, 3, 0, 15, 0]
    for a in range(8):
        for b in range(8 - a):
            for cc in range(8 - a - b):
                s = np.sum(W * c[:, 0] ** a * c[:, 1] ** b * c[:, 2] ** cc)
                assert s == pytest.approx(normal[a] * normal[b] * normal[cc], abs=1e-12)
                ref = np.sum(w * x ** a) * np.sum(w * x ** b) * np.sum(w * x ** cc)
                assert s == pytest.approx(ref, abs=1e-12)
    assert abs(np.sum(W * c[:, 2] ** 8) - 105.0) > 1.0


def test_gauss_hermite_exactness(orc):
    """sum w c^n equals the standard normal moments 1,0,1,0,3,0,15,0 for n <= 7
    (Gauss-Hermite with 4 nodes is exact to degree 7) and fails at n = 8 (105)."""
    c, W = orc.lattice(1)
    c = c[:, 0]
    normal = [1, 0, 1, 0, 3, 0, 15, 0, 105]
    for n in range(8):
        assert np.sum(W * c ** n) == pytest.approx(normal[n], abs=1e-13)
    assert abs(np.sum(W * c ** 8) - 105.0) > 1.0


def _random_pops(rng, dim, Q):
    W = orc_W(dim)
    return W * (1.0 + 0.4 * rng.uniform(-1, 1, Q))


_WCACHE = {}


def orc_W(dim):
    import oracle

    if dim not in _WCACHE:
        _WCACHE[dim] = oracle.lattice(dim)[1]
    return _WCACHE[dim]


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("order", [2, 3])
def test_grad_moment_invariance(orc, dim, order):
    """Defining condition of the regularized transformation (Sec. II.C): the projected
    populations reproduce M_0..M_order in the new frame, for arbitrary moments and frames."""
    rng = np.random.default_rng(1 + dim + 10 * order)
    Q = 4 ** dim
    for _ in range(30):
        f = _random_pops(rng, dim, Q) * rng.uniform(0.1, 10)
        u0 = rng.uniform(-3, 3, dim)
        T0 = rng.uniform(0.05, 5)
        M = orc.moments(dim, order, f, u0, T0)
        u1 = rng.uniform(-3, 3, dim)
        T1 = rng.uniform(0.05, 5)
        g = orc.grad_project(dim, order, M, u1, T1)
        M1 = orc.moments(dim, order, g, u1, T1)
        scale = np.abs(M).max()
        assert np.abs(M1 - M).max() <= 1e-12 * scale


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_grad_does_not_keep_fourth_moment(orc, dim):
    """A plausible wrong projection keeps all populations (identity). Grad order 2 must
    lose M_3 in general, and order 3 must reproduce only up to M_3."""
    rng = np.random.default_rng(7)
    Q = 4 ** dim
    f = _random_pops(rng, dim, Q)
    u, T = rng.uniform(-1, 1, dim), 0.8
    M3 = orc.moments(dim, 3, f, u, T)
    g2 = orc.grad_project(dim, 2, M3[: orc.nmom(dim, 2)], u, T)
    assert np.abs(orc.moments(dim, 3, g2, u, T) - M3).max() > 1e-3
    if dim >= 2:
        g3 = orc.grad_project(dim, 3, M3, u, T)
        # 16 populations and 10 moments (64 and 20 in 3D): not the identity
        assert np.abs(g3 - f).max() > 1e-4


def test_d1q4_grad_equals_vandermonde_solve(orc):
    """1D special case: with 4 nodes and 4 moments, the third-order Grad projection is
    the unique solution of sum_i f_i (v_i)^k = M_k, k = 0..3 (numpy linear solve)."""
    rng = np.random.default_rng(3)
    c, W = orc.lattice(1)
    c = c[:, 0]
    for _ in range(20):
        M = np.array([rng.uniform(0.5, 2), rng.uniform(-1, 1), rng.uniform(1, 3),
                      rng.uniform(-2, 2)])
        u, T = rng.uniform(-2, 2), rng.uniform(0.2, 3)
        v = math.sqrt(T) * c + u
        A = np.vstack([v ** k for k in range(4)])
        f_ref = np.linalg.solve(A, M)
        f = orc.grad_project(1, 3, M, u, T)
        assert np.abs(f - f_ref).max() <= 1e-11 * np.abs(f_ref).max()


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_equilibrium_is_fixed_point(orc, dim):
    """In its own co-moving frame the equilibrium rho W_i (Sec. II.B) has a1 = a2 = a3 = 0,
    so its projection is rho W_i itself."""
    c, W = orc.lattice(dim)
    rho, u, T = 1.7, np.array([0.4, -0.9, 0.25])[:dim], 0.6
    f = rho * W
    M = orc.moments(dim, 3, f, u, T)
    a = orc.grad_coefficients(dim, 3, M, u, T)
    assert a[0] == pytest.approx(rho, rel=1e-14)
    assert np.abs(a[1:]).max() < 1e-12
    # the equilibrium's moments are those of a Maxwellian: M2 = rho (T I + u u)
    M2 = M[1 + dim: 1 + dim + dim * dim].reshape(dim, dim)
    assert np.allclose(M2, rho * (T * np.eye(dim) + np.outer(u, u)), atol=1e-13)
    # and M3 = rho (u u u + T (u_a d_bc + u_b d_ac + u_c d_ab))
    I = np.eye(dim)
    M3 = M[1 + dim + dim * dim:].reshape(dim, dim, dim)
    M3_ref = rho * (np.einsum("a,b,c->abc", u, u, u) + T * (np.einsum("a,bc->abc", u, I)
                    + np.einsum("b,ac->abc", u, I) + np.einsum("c,ab->abc", u, I)))
    assert np.allclose(M3, M3_ref, atol=1e-13)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_grad_round_trip_and_idempotence(orc, dim):
    """Projecting Grad-form data back into its own frame returns it unchanged, and a
    round trip lambda -> lambda' -> lambda keeps the moments up to order 3."""
    rng = np.random.default_rng(11)
    Q = 4 ** dim
    f = _random_pops(rng, dim, Q)
    u0, T0 = rng.uniform(-1, 1, dim), 1.3
    g = orc.grad_project(dim, 3, orc.moments(dim, 3, f, u0, T0), u0, T0)
    g2 = orc.grad_project(dim, 3, orc.moments(dim, 3, g, u0, T0), u0, T0)
    assert np.abs(g2 - g).max() < 1e-13
    u1, T1 = rng.uniform(-1, 1, dim), 0.4
    h = orc.grad_project(dim, 3, orc.moments(dim, 3, g, u0, T0), u1, T1)
    back = orc.grad_project(dim, 3, orc.moments(dim, 3, h, u1, T1), u0, T0)
    assert np.abs(back - g).max() < 1e-12


def test_relaxation_maps_follow_definitions(orc):
    """The DUGKS variables (Sec. III.B): phi~ = phi - (dt/2)Omega, phi-bar = phi - (h/2)Omega,
    phi-bar-plus = phi + (h/2)Omega with h = dt/2, Omega = (phi_eq - phi)/tau; the update's
    collision part is the trapezoidal rule phi^{n+1} - phi^n = (dt/2)(Omega^{n+1} + Omega^n)."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        tau = rng.uniform(1e-3, 1.0)
        dt = rng.uniform(1e-4, 2.0) * tau
        h = dt / 2.0
        phi, feq = rng.uniform(0.1, 2), rng.uniform(0.1, 2)
        om = (feq - phi) / tau
        ftilde = phi - dt / 2.0 * om
        eps = dt / tau
        assert orc.phibar_plus(ftilde, feq, eps) == pytest.approx(phi + h / 2.0 * om, rel=1e-13)
        phibar = phi - h / 2.0 * om
        assert orc.face_recover(phibar, feq, eps) == pytest.approx(phi, rel=1e-13)
        # trapezoid: phi~^{n+1} = phi^{n+1} - (dt/2)Omega^{n+1} = phi^n + (dt/2)Omega^n
        assert orc.update_relax(ftilde, feq, eps) == pytest.approx(phi + dt / 2.0 * om, rel=1e-13)
    # closed forms of the coefficients (derived algebra): they sum to one
    for eps in (0.0, 0.3, 4.0, 50.0):
        a = orc.phibar_plus(1.0, 0.0, eps)
        b = orc.phibar_plus(0.0, 1.0, eps)
        assert a == pytest.approx((2 - eps / 2) / (2 + eps), abs=1e-15)
        assert b == pytest.approx((1.5 * eps) / (2 + eps), abs=1e-15)
        assert a + b == pytest.approx(1.0, abs=1e-15)


def test_limiters(orc):
    """Van Leer (harmonic) and minmod slope limiters: zero at extrema, symmetric, exact on
    linear data, bounded by twice (Van Leer) or once (minmod) the smaller difference."""
    rng = np.random.default_rng(2)
    for kind in ("vanleer", "minmod"):
        assert orc.limiter(kind, 1.0, -2.0) == 0.0
        assert orc.limiter(kind, 0.0, 2.0) == 0.0
        assert orc.limiter(kind, 0.7, 0.7) == pytest.approx(0.7)
        for _ in range(100):
            a, b = rng.uniform(-3, 3, 2)
            s = orc.limiter(kind, a, b)
            assert s == pytest.approx(orc.limiter(kind, b, a))
            assert orc.limiter(kind, -a, -b) == pytest.approx(-s)
            if a * b > 0:
                assert abs(s) <= (2.0 if kind == "vanleer" else 1.0) * min(abs(a), abs(b)) + 1e-15
                assert np.sign(s) == np.sign(a)
    assert orc.limiter("vanleer", 1.0, 3.0) == pytest.approx(1.5)
    assert orc.limiter("minmod", 1.0, 3.0) == pytest.approx(1.0)
