"""Pins of the oracle's semi-Lagrangian realization (Sec. III.A) in 1D (the 2D pins are
in test_oracle_sl2d.py): frame iteration of the advection from the departure points,
interpolating cubic kernel with a clipping limiter over the cell centres, BGK collision."""
import math

import numpy as np
import pytest

import exact_riemann as ER
from paper_2203_05477_amd import workloads as W


def _sl(cfg):
    return dict(cfg, scheme="sl")


def test_uniform_flow_stays_uniform(orc):
    cfg, f = W.uniform(1, 16, rho=1.3, u=(0.7, 0.0), p=0.9, tol=1e-13)
    s = orc.Sim(_sl(cfg), f["rho"], f["ux"], None, f["p"])
    for _ in range(5):
        s.step()
    r, u, _, T = s.fields()
    assert np.abs(r - 1.3).max() < 1e-14 and np.abs(u - 0.7).max() < 1e-14
    assert np.abs(T - 0.9 / 1.3).max() < 1e-14


def test_smooth_wave_second_order(orc):
    """A density wave advected in a uniform-pressure flow (periodic): the cubic kernel
    makes the advection second order at least (a linear kernel, or a departure point at
    half the step, would show first order or a wrong phase)."""
    errs = []
    for nx in (32, 64, 128):
        cfg = W.base_config(1, nx, cfl=0.3, mu=1e-6, tol=1e-12, bc=("periodic",) * 4)
        x, _ = W.cell_centres(cfg)
        dx = 1.0 / nx
        rho = 1.0 + 0.2 * (np.cos(2 * np.pi * (x - dx / 2)) - np.cos(2 * np.pi * (x + dx / 2))) / (2 * np.pi * dx)
        s = orc.Sim(_sl(cfg), rho, np.full(nx, 1.0), None, np.full(nx, 1.0))
        while s.t < 0.25 * (1 - 1e-12):
            s.step(0.25)
        r, _, _, _ = s.fields()
        ex = 1.0 + 0.2 * (np.cos(2 * np.pi * (x - dx / 2 - 0.25)) - np.cos(2 * np.pi * (x + dx / 2 - 0.25))) / (2 * np.pi * dx)
        errs.append(np.abs(r - ex).mean())
    assert math.log2(errs[0] / errs[1]) > 1.7 and math.log2(errs[1] / errs[2]) > 1.7, errs


def test_shock_tube_against_exact_and_not_conservative(orc):
    """The shock tube: small L1 error against the exact Riemann solution, falling under
    refinement; the total mass is not conserved (the scheme is not in flux form, the
    paper's reason for the finite-volume scheme), but its drift shrinks with the cell
    size, about linearly."""
    errs, drifts = [], []
    for nx in (100, 200, 400):
        cfg, f = W.shock_tube(nx, tol=1e-10)
        s = orc.Sim(_sl(cfg), f["rho"], f["ux"], None, f["p"])
        m0 = s.conserved()[0].sum()
        while s.t < 0.2 * (1 - 1e-12):
            s.step(0.2)
        U = s.conserved()
        ex = ER.cell_average((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, np.linspace(0, 1, nx + 1), 0.5, 0.2)
        errs.append(np.abs(U[0] - ex[0]).sum() / np.abs(ex[0]).sum())
        drifts.append(abs(U[0].sum() - m0) / m0)
    assert errs[2] < errs[1] < errs[0] < 0.03
    assert drifts[0] > 1e-4 and drifts[2] < drifts[1] < drifts[0]
    assert drifts[0] / drifts[2] > 2.0


def test_mirror_symmetry(orc):
    """A state symmetric under x -> 1 - x stays symmetric (rho, T even, u odd)."""
    cfg = W.base_config(1, 40, cfl=0.3, tol=1e-13, bc=("outflow",) * 4)
    x, _ = W.cell_centres(cfg)
    rho = 1.0 + 0.5 * np.exp(-40 * (x - 0.5) ** 2)
    p = 1.0 + 2.0 * np.exp(-40 * (x - 0.5) ** 2)
    s = orc.Sim(_sl(cfg), rho, 0.3 * np.sin(2 * np.pi * (x - 0.5)), None, p)
    for _ in range(10):
        s.step()
    r, u, _, T = s.fields()
    assert np.abs(r - r[::-1]).max() < 1e-13
    assert np.abs(u + u[::-1]).max() < 1e-13
    assert np.abs(T - T[::-1]).max() < 1e-13


def test_three_dimensions_are_not_built(orc):
    cfg, f = W.random_smooth_3d(6, 5, 4, seed=1)
    with pytest.raises(Exception):
        orc.Sim(_sl(cfg), f["rho"], f["ux"], f["uy"], f["p"], uz=f["uz"])
