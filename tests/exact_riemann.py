"""Exact solution of the 1D Riemann problem for an ideal gas (test reference only).

Written from the mathematics of the Euler equations: across a shock the
Rankine-Hugoniot relations hold, across a rarefaction the Riemann invariant and
the isentrope hold; the star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0,
with f_K the velocity change across the K-wave as a function of the star
pressure. A safeguarded Newton iteration finds p*. Vacuum generation
(2 (c_L + c_R)/(gamma - 1) <= u_R - u_L) is sampled as two rarefactions into
vacuum. The paper compares its shock tubes with such a solver (Sec. IV.A-B).
"""
from __future__ import annotations

import math

import numpy as np


def _wave(p, rho_k, p_k, g):
    """velocity change across the K wave and its derivative w.r.t. the star pressure"""
    c_k = math.sqrt(g * p_k / rho_k)
    if p > p_k:  # shock
        A = 2.0 / ((g + 1.0) * rho_k)
        B = (g - 1.0) / (g + 1.0) * p_k
        q = math.sqrt(A / (p + B))
        return (p - p_k) * q, q * (1.0 - 0.5 * (p - p_k) / (p + B))
    # rarefaction
    e = (g - 1.0) / (2.0 * g)
    r = (p / p_k) ** e
    return 2.0 * c_k / (g - 1.0) * (r - 1.0), 1.0 / (rho_k * c_k) * (p / p_k) ** (-(g + 1.0) / (2.0 * g))


def star_state(left, right, gamma):
    """(p*, u*) of the Riemann problem, or None when the waves open a vacuum."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        return None
    du = ur - ul

    def F(p):
        a, da = _wave(p, rl, pl, g)
        b, db = _wave(p, rr, pr, g)
        return a + b + du, da + db

    # bracket: F is increasing in p, F(0+) < 0 when there is no vacuum
    lo, hi = 0.0, max(pl, pr)
    while F(hi)[0] < 0.0:
        lo, hi = hi, hi * 2.0
    p = 0.5 * (lo + hi)
    for _ in range(200):
        val, der = F(p)
        if val > 0.0:
            hi = p
        else:
            lo = p
        step = p - val / der
        p_new = step if lo < step < hi else 0.5 * (lo + hi)
        if abs(p_new - p) <= 1e-15 * max(p, 1e-300) or hi - lo <= 1e-15 * hi:
            p = p_new
            break
        p = p_new
    a, _ = _wave(p, rl, pl, g)
    b, _ = _wave(p, rr, pr, g)
    u = 0.5 * (ul + ur) + 0.5 * (b - a)
    return p, u


def residual(left, right, gamma, p):
    a, _ = _wave(p, left[0], left[2], gamma)
    b, _ = _wave(p, right[0], right[2], gamma)
    return a + b + (right[1] - left[1])


def sample(left, right, gamma, xi):
    """Primitive state (rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    xi = np.asarray(xi, dtype=np.float64)
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    out = np.zeros((3,) + xi.shape)
    st = star_state(left, right, gamma)
    gm1, gp1 = g - 1.0, g + 1.0

    def left_fan(s):
        u = 2.0 / gp1 * (cl + gm1 / 2.0 * ul + s)
        c = 2.0 / gp1 * (cl + gm1 / 2.0 * (ul - s))
        rho = rl * (c / cl) ** (2.0 / gm1)
        return rho, u, pl * (c / cl) ** (2.0 * g / gm1)

    def right_fan(s):
        u = 2.0 / gp1 * (-cr + gm1 / 2.0 * ur + s)
        c = 2.0 / gp1 * (cr - gm1 / 2.0 * (ur - s))
        rho = rr * (c / cr) ** (2.0 / gm1)
        return rho, u, pr * (c / cr) ** (2.0 * g / gm1)

    for idx, s in np.ndenumerate(xi):
        if st is None:  # two rarefactions into vacuum
            sl_head, sl_tail = ul - cl, ul + 2.0 * cl / gm1
            sr_head, sr_tail = ur + cr, ur - 2.0 * cr / gm1
            if s <= sl_head:
                v = (rl, ul, pl)
            elif s < sl_tail:
                v = left_fan(s)
            elif s <= sr_tail:
                v = (0.0, 0.5 * (sl_tail + sr_tail), 0.0)
            elif s < sr_head:
                v = right_fan(s)
            else:
                v = (rr, ur, pr)
            out[(slice(None),) + idx] = v
            continue
        ps, us = st
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sL = ul - cl * math.sqrt(gp1 / (2 * g) * ps / pl + gm1 / (2 * g))
                if s <= sL:
                    v = (rl, ul, pl)
                else:
                    rho = rl * (ps / pl + gm1 / gp1) / (gm1 / gp1 * ps / pl + 1.0)
                    v = (rho, us, ps)
            else:
                cs = cl * (ps / pl) ** (gm1 / (2 * g))
                if s <= ul - cl:
                    v = (rl, ul, pl)
                elif s >= us - cs:
                    v = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    v = left_fan(s)
        else:
            if ps > pr:  # right shock
                sR = ur + cr * math.sqrt(gp1 / (2 * g) * ps / pr + gm1 / (2 * g))
                if s >= sR:
                    v = (rr, ur, pr)
                else:
                    rho = rr * (ps / pr + gm1 / gp1) / (gm1 / gp1 * ps / pr + 1.0)
                    v = (rho, us, ps)
            else:
                cs = cr * (ps / pr) ** (gm1 / (2 * g))
                if s >= ur + cr:
                    v = (rr, ur, pr)
                elif s <= us + cs:
                    v = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    v = right_fan(s)
        out[(slice(None),) + idx] = v
    return out


def cell_average(left, right, gamma, x_edges, x0, t, sub=16):
    """Cell averages of (rho, rho u, rho E) of the exact solution over the given cells
    (midpoint sub-sampling), for L1 error measurements."""
    x_edges = np.asarray(x_edges, dtype=np.float64)
    n = x_edges.size - 1
    U = np.zeros((3, n))
    for k in range(sub):
        xs = x_edges[:-1] + (k + 0.5) / sub * (x_edges[1:] - x_edges[:-1])
        r, u, p = sample(left, right, gamma, (xs - x0) / t)
        U[0] += r
        U[1] += r * u
        U[2] += p / (gamma - 1.0) + 0.5 * r * u * u
    return U / sub
