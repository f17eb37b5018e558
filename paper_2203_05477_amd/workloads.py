"""Seeded, synthetic workloads for the finite-volume PonD step.

This module only builds initial primitive fields (rho, ux, uy, p) on a uniform
grid and the configuration dict that goes with them. It holds none of the
method's arithmetic, imports neither the GPU binding nor the oracle, and serves
both sides of every parity test, the benchmark and users alike.

The set-ups take the shapes, states and boundary conditions of the problems the
paper prints (Sec. IV): Sod-type shock tubes, the double Mach reflection, a
shocked density interface and the Mach-80 jet, plus a batch of random shock
tubes. All values are in units with gas constant 1 (p = rho T).
"""
from __future__ import annotations

import math

import numpy as np

# frame-iteration tolerances by use: the tight value for parity against the oracle,
# production values per precision (the learned seed uses the same as the plain one)
TOL_PARITY = 1e-13
TOL_FP64 = 1e-10
TOL_FP32 = 1e-5


def base_config(dim, nx, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, gamma=1.4, cfl=0.2,
                mu=1e-3, tol=TOL_PARITY, max_iter=32, limiter="vanleer",
                bc=("outflow", "outflow", "outflow", "outflow")):
    z = [[0.0] * 4 for _ in range(4)]
    return {
        "dim": dim, "nx": nx, "ny": ny if dim >= 2 else 1,
        "x0": x0, "x1": x1, "y0": y0, "y1": y1,
        "gamma": gamma, "cfl": cfl, "mu": mu, "tol": tol, "max_iter": max_iter,
        "limiter": limiter, "bc": list(bc),
        "bc_state": [list(r) for r in z], "bc_alt": [list(r) for r in z],
        "bc_param": [list(r) for r in z],
    }


def base_config_3d(nx, ny, nz, x0=0.0, x1=1.0, y0=0.0, y1=1.0, z0=0.0, z1=1.0, bc=("periodic",) * 6,
                   **kw):
    """A 3D box (D3Q64): sides west, east, south, north, bottom, top; the periodic, outflow
    and reflecting kinds."""
    cfg = base_config(3, nx, ny, x0=x0, x1=x1, y0=y0, y1=y1, bc=tuple(bc[:4]), **kw)
    cfg["nz"], cfg["z0"], cfg["z1"] = nz, z0, z1
    cfg["bc"] = list(bc)
    return cfg


def cell_centres_3d(cfg):
    """X, Y, Z of every cell, index i + nx (j + ny k)."""
    ax = []
    for n, a, b in (("nx", "x0", "x1"), ("ny", "y0", "y1"), ("nz", "z0", "z1")):
        h = (cfg[b] - cfg[a]) / cfg[n]
        ax.append(cfg[a] + (np.arange(cfg[n]) + 0.5) * h)
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def random_smooth_3d(nx, ny, nz, seed=0, amp=0.3, bc="periodic", **kw):
    """Periodic, smooth random fields in a unit box (a few Fourier modes per field)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cfg = base_config_3d(nx, ny, nz, bc=(bc,) * 6, **kw)
    X, Y, Z = cell_centres_3d(cfg)

    def field(base, a):
        out = np.full(X.shape, base, dtype=np.float64)
        for _ in range(3):
            k = rng.integers(0, 3, 3)
            k[rng.integers(0, 3)] += 1
            ph = rng.uniform(0, 2 * np.pi)
            out += a * rng.uniform(-1, 1) * np.sin(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
        return out

    cfg["name"] = "random_smooth_3d"
    return cfg, {"rho": field(1.0, amp), "ux": field(0.0, amp), "uy": field(0.0, amp),
                 "uz": field(0.0, amp), "p": field(1.0, amp)}


def riemann_3d(left, right, axis=0, n=100, nt=2, xi=0.5, gamma=1.4, cfl=0.5, mu=1e-3,
               tol=TOL_PARITY, max_iter=32):
    """A 1D Riemann problem along `axis` (0, 1, 2) of a 3D box: n cells of [0, 1] along it,
    outflow at its ends; nt cells (periodic) across; left = (rho, u_n, p) below xi."""
    ns = [nt, nt, nt]
    ns[axis] = n
    bc = ["periodic"] * 6
    bc[2 * axis], bc[2 * axis + 1] = "outflow", "outflow"
    cfg = base_config_3d(*ns, bc=bc, gamma=gamma, cfl=cfl, mu=mu, tol=tol, max_iter=max_iter)
    C = cell_centres_3d(cfg)[axis]
    L = C < xi
    vel = [np.zeros(C.size) for _ in range(3)]
    vel[axis] = np.where(L, left[1], right[1]).astype(np.float64)
    cfg["name"] = "riemann_3d"
    return cfg, {"rho": np.where(L, left[0], right[0]).astype(np.float64), "ux": vel[0],
                 "uy": vel[1], "uz": vel[2], "p": np.where(L, left[2], right[2]).astype(np.float64)}


def cell_centres(cfg):
    dx = (cfg["x1"] - cfg["x0"]) / cfg["nx"]
    x = cfg["x0"] + (np.arange(cfg["nx"]) + 0.5) * dx
    if cfg["dim"] == 1:
        return x, None
    dy = (cfg["y1"] - cfg["y0"]) / cfg["ny"]
    y = cfg["y0"] + (np.arange(cfg["ny"]) + 0.5) * dy
    X, Y = np.meshgrid(x, y)  # row-major: index = i + nx * j
    return X.ravel(), Y.ravel()


def riemann_1d(left, right, nx=400, x0=0.0, x1=1.0, xi=0.5, gamma=1.4, cfl=0.5, mu=1e-3,
               tol=TOL_PARITY, max_iter=32, bc=("outflow", "outflow")):
    """A 1D Riemann problem: state `left` = (rho, u, p) for x_c < xi, `right` beyond."""
    cfg = base_config(1, nx, x0=x0, x1=x1, gamma=gamma, cfl=cfl, mu=mu, tol=tol,
                      max_iter=max_iter, bc=(bc[0], bc[1], "outflow", "outflow"))
    x, _ = cell_centres(cfg)
    L = x < xi
    rho = np.where(L, left[0], right[0]).astype(np.float64)
    u = np.where(L, left[1], right[1]).astype(np.float64)
    p = np.where(L, left[2], right[2]).astype(np.float64)
    cfg["name"] = "riemann_1d"
    cfg["riemann"] = {"left": tuple(left), "right": tuple(right), "xi": xi}
    return cfg, {"rho": rho, "ux": u, "uy": None, "p": p}


def shock_tube(nx=400, **kw):
    """1D shock tube on [0,1], interface 0.5, (1, 0, 1) | (0.125, 0, 0.1), gamma 1.4,
    CFL 0.5, run to t = 0.2 (Sod-type, Sec. IV.A.1 with the textbook pressures)."""
    kw.setdefault("cfl", 0.5)
    cfg, f = riemann_1d((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), nx=nx, **kw)
    cfg["name"] = "shock_tube"
    cfg["t_end"] = 0.2
    return cfg, f


# further 1D Riemann problems printed in Sec. IV.A-B and IV.C.5: (left, right, xi, domain,
# gamma, t_end, the paper's resolution L, viscosity mu)
#
# The paper asks only for a viscosity low enough that the results no longer change. With
# tau = mu/p, eps = dt p/mu sets how close each gas is to the Euler limit, and the pressures
# of these problems span 1e-10..1e3: Le Blanc's hot gas (p = 0.067) is still far from it at
# mu = 1e-4 (the step loses positivity at some resolutions), and the strong shock tube's
# (p = 1000) is so far past it at mu = 1e-5 that the step breaks down at once. Each case
# takes a mu inside the window where it runs at every resolution from 100 cells up and its
# L1 error moves by a few per cent at most between neighbouring values.
RIEMANN_CASES = {
    "lax": ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571), 0.5, (0.0, 1.0), 1.4, 0.14, 600, 1e-5),
    "strong_shock": ((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01), 0.5, (0.0, 1.0), 1.4, 0.012, 800,
                     1e-4),
    "double_rarefaction": ((1.0, -2.0, 0.1), (1.0, 2.0, 0.1), 0.5, (0.0, 1.0), 1.4, 0.1, 800,
                           1e-4),
    "le_blanc": ((1.0, 0.0, 2.0 / 3.0 * 1e-1), (1e-3, 0.0, 2.0 / 3.0 * 1e-10), 3.0, (0.0, 9.0),
                 5.0 / 3.0, 6.0, 4000, 1e-5),
    "jet_1d": ((5.0, 30.0, 0.4127), (0.5, 0.0, 0.4127), 0.1, (0.0, 2.0), 5.0 / 3.0, 0.06, 1500,
               1e-4),
}


def riemann_case(name, nx=None, cfl=0.2, mu=None, **kw):
    """One of the printed 1D Riemann problems, outflow at both ends, at the paper's
    resolution unless `nx` is given; `cfg["t_end"]` is the printed final time."""
    left, right, xi, (a, b), gamma, t_end, L, mu0 = RIEMANN_CASES[name]
    cfg, f = riemann_1d(left, right, nx=nx or L, x0=a, x1=b, xi=xi, gamma=gamma, cfl=cfl,
                        mu=mu0 if mu is None else mu, **kw)
    cfg["name"] = name
    cfg["t_end"] = t_end
    return cfg, f


def rankine_hugoniot(rho1, p1, mach, gamma):
    """Post-shock (rho2, p2, normal velocity jump) for a shock of Mach `mach` moving into
    gas at rest (rho1, p1) -- normal-shock relations, used only to build set-ups."""
    g = gamma
    m2 = mach * mach
    rho2 = rho1 * (g + 1.0) * m2 / ((g - 1.0) * m2 + 2.0)
    p2 = p1 * (1.0 + 2.0 * g / (g + 1.0) * (m2 - 1.0))
    c1 = math.sqrt(g * p1 / rho1)
    du = mach * c1 * (1.0 - rho1 / rho2)
    return rho2, p2, du


def blast_waves(nx=1600, mu=1e-4, tol=TOL_PARITY, max_iter=32):
    """Two interacting blast waves (Sec. IV.B): [0,1], reflecting ends, rho = 1, u = 0 and
    p = 1000 | 0.01 | 100 split at x = 0.1 and 0.9 (cell-centre test), gamma 1.4, CFL 0.2,
    to t = 0.038 (the paper's 1,600 points). mu = 1e-4: at 1e-5 the 1000 | 0.01 jump is
    too far past the Euler limit at the first step (as for the strong shock tube)."""
    cfg = base_config(1, nx, cfl=0.2, mu=mu, tol=tol, max_iter=max_iter, bc=("reflect",) * 4)
    x, _ = cell_centres(cfg)
    cfg["name"] = "blast_waves"
    cfg["t_end"] = 0.038
    p = np.where(x < 0.1, 1000.0, np.where(x < 0.9, 0.01, 100.0))
    return cfg, {"rho": np.ones(nx), "ux": np.zeros(nx), "uy": None, "p": p}


def explosion_box(n=256, cfl=0.2, mu=1e-3, tol=TOL_PARITY, max_iter=32):
    """Explosion in a closed box (Sec. IV.C): [0,1]^2, n x n cells (the paper's 256),
    reflecting walls; (rho, u, p) = (5, 0, 5) inside the circle of radius 0.3 around
    (0.4, 0.4) (cell-centre test), (1, 0, 1) outside; gamma 1.4; run to t = 0.5."""
    cfg = base_config(2, n, n, cfl=cfl, mu=mu, tol=tol, max_iter=max_iter, bc=("reflect",) * 4)
    x, y = cell_centres(cfg)
    inside = (x - 0.4) ** 2 + (y - 0.4) ** 2 < 0.3 ** 2
    cfg["name"] = "explosion_box"
    cfg["t_end"] = 0.5
    v = np.where(inside, 5.0, 1.0)
    return cfg, {"rho": v.copy(), "ux": np.zeros(v.size), "uy": np.zeros(v.size), "p": v.copy()}


def explosion_box_3d(n=128, cfl=0.2, mu=1e-3, tol=TOL_PARITY, max_iter=32):
    """The explosion in a closed box (Sec. IV.C) carried to three dimensions: [0,1]^3, n^3
    cells, reflecting walls on all six sides; (rho, u, p) = (5, 0, 5) inside the sphere of
    radius 0.3 around (0.4, 0.4, 0.4) (cell-centre test), (1, 0, 1) outside; gamma 1.4. The
    paper's experiments are two-dimensional; this is the same set-up on the D3Q64 lattice."""
    cfg = base_config_3d(n, n, n, cfl=cfl, mu=mu, tol=tol, max_iter=max_iter, bc=("reflect",) * 6)
    X, Y, Z = cell_centres_3d(cfg)
    inside = (X - 0.4) ** 2 + (Y - 0.4) ** 2 + (Z - 0.4) ** 2 < 0.3 ** 2
    cfg["name"] = "explosion_box_3d"
    v = np.where(inside, 5.0, 1.0)
    z = np.zeros(v.size)
    return cfg, {"rho": v.copy(), "ux": z, "uy": z.copy(), "uz": z.copy(), "p": v.copy()}


def double_mach(nx=1920, ny=480, mach=10.0, gamma=1.4, cfl=0.2, mu=1e-3, tol=TOL_PARITY,
                max_iter=32):
    """Mach-10 shock meeting a 30 degree wall (Sec. IV.C.4): [0,4]x[0,1]; shock through
    (1/6, 0) inclined 60 degrees to the x axis; pre-shock (1.4, 0, 0, 1); post-shock
    from the normal-shock relations; bottom fixed post-shock for x < 1/6 and reflecting
    beyond; left fixed post-shock; right outflow; top follows the moving shock."""
    rho1, p1 = 1.4, 1.0
    rho2, p2, du = rankine_hugoniot(rho1, p1, mach, gamma)
    ang = math.radians(30.0)
    u2 = (du * math.cos(ang), -du * math.sin(ang))
    post = [rho2, u2[0], u2[1], p2]
    pre = [rho1, 0.0, 0.0, p1]
    xw = 1.0 / 6.0
    inv_tan = 1.0 / math.sqrt(3.0)
    c1 = math.sqrt(gamma * p1 / rho1)
    speed_x = mach * c1 / math.sin(math.radians(60.0))  # x-speed of the shock trace
    cfg = base_config(2, nx, ny, 0.0, 4.0, 0.0, 1.0, gamma=gamma, cfl=cfl, mu=mu, tol=tol,
                      max_iter=max_iter,
                      bc=("fixed", "outflow", "split_fixed_reflect", "moving_shock"))
    cfg["bc_state"][0] = list(post)
    cfg["bc_state"][2] = list(post)
    cfg["bc_param"][2] = [xw, 0.0, 0.0, 0.0]
    cfg["bc_state"][3] = list(post)
    cfg["bc_alt"][3] = list(pre)
    # x_s(y, t) = xw + (y + v t)/sqrt(3), with v = speed_x * sqrt(3) = 20 for Mach 10
    cfg["bc_param"][3] = [xw, inv_tan, speed_x * math.sqrt(3.0), 0.0]
    cfg["name"] = "double_mach"
    X, Y = cell_centres(cfg)
    behind = X < xw + Y * inv_tan
    fields = {
        "rho": np.where(behind, post[0], pre[0]),
        "ux": np.where(behind, post[1], pre[1]),
        "uy": np.where(behind, post[2], pre[2]),
        "p": np.where(behind, post[3], pre[3]),
    }
    cfg["post"] = post
    cfg["pre"] = pre
    return cfg, fields


def shocked_interface(nx=2048, ny=512, mach=2.0, density_ratio=3.0, amplitude=0.05,
                      gamma=1.4, cfl=0.2, mu=1e-3, tol=TOL_FP32, max_iter=32):
    """Shock of Mach `mach` in light gas (1, 0, 0, 1) hitting a heavy/light interface
    (density ratio 3) at x_I(y) = 1 + a cos(2 pi y) on [0,4]x[0,1], periodic in y;
    left fixed post-shock inflow, right outflow (stand-in for Sec. IV.C.3)."""
    rho1, p1 = 1.0, 1.0
    rho2, p2, du = rankine_hugoniot(rho1, p1, mach, gamma)
    post = [rho2, du, 0.0, p2]
    cfg = base_config(2, nx, ny, 0.0, 4.0, 0.0, 1.0, gamma=gamma, cfl=cfl, mu=mu, tol=tol,
                      max_iter=max_iter, bc=("fixed", "outflow", "periodic", "periodic"))
    cfg["bc_state"][0] = list(post)
    cfg["name"] = "shocked_interface"
    X, Y = cell_centres(cfg)
    xI = 1.0 + amplitude * np.cos(2.0 * np.pi * Y)
    rho = np.where(X < xI, rho1, rho1 * density_ratio)
    rho = np.where(X < 0.5, post[0], rho)
    ux = np.where(X < 0.5, post[1], 0.0)
    p = np.where(X < 0.5, post[3], p1)
    return cfg, {"rho": rho, "ux": ux, "uy": np.zeros_like(rho), "p": p}


def jet(nx=2048, ny=2048, gamma=5.0 / 3.0, cfl=0.2, mu=1e-3, tol=TOL_FP32, max_iter=32,
        width=0.1, speed=30.0, x1=1.0):
    """Mach-80 jet (Sec. IV.C.5): [0,x1]x[-0.5,0.5] (the paper's domain has x1 = 2 on
    [1000,500] cells; x1 = 1 keeps square cells on a square grid); ambient (0.5, 0, 0,
    0.4127); left boundary fixed jet (5, speed = 30, 0, 0.4127) for |y| <= width/2, fixed
    ambient elsewhere; other sides outflow; gamma 5/3."""
    amb = [0.5, 0.0, 0.0, 0.4127]
    jet_state = [5.0, float(speed), 0.0, 0.4127]
    cfg = base_config(2, nx, ny, 0.0, x1, -0.5, 0.5, gamma=gamma, cfl=cfl, mu=mu, tol=tol,
                      max_iter=max_iter, bc=("fixed_window", "outflow", "outflow", "outflow"))
    cfg["bc_state"][0] = list(amb)
    cfg["bc_alt"][0] = list(jet_state)
    cfg["bc_param"][0] = [-0.5 * width, 0.5 * width, 0.0, 0.0]
    cfg["name"] = "jet"
    n = nx * ny
    return cfg, {"rho": np.full(n, amb[0]), "ux": np.zeros(n), "uy": np.zeros(n),
                 "p": np.full(n, amb[3])}


def strip_2d(cfg1, fields1, ny=4):
    """A 1D workload embedded in 2D: the same cells in x, `ny` identical rows periodic in y
    (square cells), the x boundary conditions and states kept; a y-uniform 2D flow."""
    nx = cfg1["nx"]
    dx = (cfg1["x1"] - cfg1["x0"]) / nx
    cfg = base_config(2, nx, ny, cfg1["x0"], cfg1["x1"], 0.0, ny * dx, gamma=cfg1["gamma"],
                      cfl=cfg1["cfl"], mu=cfg1["mu"], tol=cfg1["tol"], max_iter=cfg1["max_iter"],
                      limiter=cfg1.get("limiter", "vanleer"),
                      bc=(cfg1["bc"][0], cfg1["bc"][1], "periodic", "periodic"))
    for k in range(2):
        cfg["bc_state"][k] = list(cfg1["bc_state"][k])
        cfg["bc_alt"][k] = list(cfg1["bc_alt"][k])
        cfg["bc_param"][k] = list(cfg1["bc_param"][k])
    cfg["name"] = cfg1.get("name", "strip") + "_strip"
    rep = lambda a: np.tile(np.asarray(a, dtype=np.float64), ny)  # noqa: E731
    return cfg, {"rho": rep(fields1["rho"]), "ux": rep(fields1["ux"]), "uy": np.zeros(nx * ny),
                 "p": rep(fields1["p"])}


def uniform(dim, nx, ny=1, rho=1.0, u=(0.3, -0.2), p=0.7, bc="periodic", **kw):
    cfg = base_config(dim, nx, ny, bc=(bc,) * 4, **kw)
    n = nx * (ny if dim == 2 else 1)
    cfg["name"] = "uniform"
    return cfg, {"rho": np.full(n, float(rho)), "ux": np.full(n, float(u[0])),
                 "uy": np.full(n, float(u[1])) if dim == 2 else None, "p": np.full(n, float(p))}


def random_smooth(dim, nx, ny=1, seed=0, amp=0.3, bc="periodic", **kw):
    """Periodic, smooth random fields (a few Fourier modes) -- for conservation tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cfg = base_config(dim, nx, ny, bc=(bc,) * 4, **kw)
    X, Y = cell_centres(cfg)
    if Y is None:
        Y = np.zeros_like(X)

    def field(base, a):
        out = np.full(X.shape, base, dtype=np.float64)
        for _ in range(3):
            kx, ky = rng.integers(1, 4), (rng.integers(0, 3) if dim == 2 else 0)
            ph = rng.uniform(0, 2 * np.pi)
            out += a * rng.uniform(-1, 1) * np.sin(2 * np.pi * (kx * X + ky * Y) + ph)
        return out

    rho = field(1.0, amp * 0.5)
    ux = field(0.2, amp)
    uy = field(-0.1, amp) if dim == 2 else None
    p = field(1.0, amp * 0.5)
    cfg["name"] = "random_smooth"
    return cfg, {"rho": rho, "ux": ux, "uy": uy, "p": p}


# --------------------------------------------------------------------------------------
# batched 1D shock tubes
# --------------------------------------------------------------------------------------

TUBES_SEED = 220305477


def tube_batch(n_tubes=4096, seed=TUBES_SEED, len_lo=200, len_hi=4000, gamma=1.4, cfl=0.2,
               mu=1e-3, tol=TOL_FP32, max_iter=32, rho_decades=5.0, p_decades=6.0, mach=5.0):
    """Independent 1D shock tubes on [0,1] with the interface at 0.5 and outflow ends.
    Drawn in this order from PCG64(seed): cell count N ~ integers[len_lo, len_hi];
    density ratio 10^U[0,rho_decades); pressure ratio 10^U[0,p_decades); Mach numbers
    M_L, M_R ~ U[-mach, mach] (defaults 5, 6 and 5);
    two fair coins for the dense and the high-pressure side. The dense side has
    rho = 1, the other 1/ratio; the high side p = 1, the other 1/ratio;
    u = M sqrt(gamma p / rho). Tubes whose exact solution would open a vacuum
    (2 (c_L + c_R)/(gamma - 1) <= u_R - u_L) are drawn again."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lens, states = [], []
    while len(lens) < n_tubes:
        N = int(rng.integers(len_lo, len_hi, endpoint=True))
        r_rho = 10.0 ** rng.uniform(0.0, rho_decades)
        r_p = 10.0 ** rng.uniform(0.0, p_decades)
        ML, MR = rng.uniform(-mach, mach), rng.uniform(-mach, mach)
        dense_left = rng.integers(0, 2) == 1
        high_left = rng.integers(0, 2) == 1
        rhoL, rhoR = (1.0, 1.0 / r_rho) if dense_left else (1.0 / r_rho, 1.0)
        pL, pR = (1.0, 1.0 / r_p) if high_left else (1.0 / r_p, 1.0)
        cL, cR = math.sqrt(gamma * pL / rhoL), math.sqrt(gamma * pR / rhoR)
        uL, uR = ML * cL, MR * cR
        if 2.0 * (cL + cR) / (gamma - 1.0) <= uR - uL:
            continue
        lens.append(N)
        states.append(((rhoL, uL, pL), (rhoR, uR, pR)))
    lens = np.asarray(lens, dtype=np.int32)
    offs = np.zeros(n_tubes + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lens)
    total = int(offs[-1])
    rho = np.empty(total); u = np.empty(total); p = np.empty(total)
    for k in range(n_tubes):
        N = int(lens[k])
        x = (np.arange(N) + 0.5) / N
        L = x < 0.5
        (a, b) = states[k]
        sl = slice(int(offs[k]), int(offs[k + 1]))
        rho[sl] = np.where(L, a[0], b[0])
        u[sl] = np.where(L, a[1], b[1])
        p[sl] = np.where(L, a[2], b[2])
    cfg = base_config(1, 0, gamma=gamma, cfl=cfl, mu=mu, tol=tol, max_iter=max_iter)
    cfg["name"] = "tube_batch"
    cfg["lengths"] = lens
    cfg["offsets"] = offs
    cfg["states"] = states
    return cfg, {"rho": rho, "ux": u, "uy": None, "p": p}


def tube_config(batch_cfg, k):
    """Single-tube configuration of tube k of a batch (for the oracle)."""
    N = int(batch_cfg["lengths"][k])
    cfg = base_config(1, N, gamma=batch_cfg["gamma"], cfl=batch_cfg["cfl"], mu=batch_cfg["mu"],
                      tol=batch_cfg["tol"], max_iter=batch_cfg["max_iter"])
    cfg["name"] = f"tube{k}"
    return cfg


def tube_fields(batch_cfg, fields, k):
    o = batch_cfg["offsets"]
    sl = slice(int(o[k]), int(o[k + 1]))
    return {"rho": fields["rho"][sl], "ux": fields["ux"][sl], "uy": None, "p": fields["p"][sl]}
