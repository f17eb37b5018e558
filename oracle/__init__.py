"""Python access to the FP64 CPU oracle of the finite-volume PonD step.

TEST INFRASTRUCTURE: the plain, slow reference that the HIP library is checked
against (Kallikounis, Dorschner & Karlin, Sec. III.B). Only ``tests/``, the smoke
check and the CPU-baseline leg of ``bench.py`` may import this package. It shares
no code with the GPU library and never imports it.

Configurations are the plain dicts produced by the workload generators
(keys: dim, nx, ny, x0, x1, y0, y1, gamma, cfl, mu, limiter, tol, max_iter, bc,
bc_state, bc_alt, bc_param, and optionally regularization and scheme); boundary kinds,
limiters, regularizations and schemes are given by name.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pond_oracle.c")
LIB_PATH = os.path.join(_HERE, "liborc.so")

BC_KIND = {
    "periodic": 0,
    "outflow": 1,
    "reflect": 2,
    "fixed": 3,
    "fixed_window": 4,
    "split_fixed_reflect": 5,
    "moving_shock": 6,
}
LIMITER = {"vanleer": 0, "minmod": 1}
REGULARIZATION = {"grad": 0, "eq": 1}
SCHEME = {"fv": 0, "sl": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-fopenmp", "-fno-fast-math", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double),
        ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("mu", ctypes.c_double),
        ("limiter", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
        ("bc", ctypes.c_int * 4),
        ("bc_state", (ctypes.c_double * 4) * 4),
        ("bc_alt", (ctypes.c_double * 4) * 4),
        ("bc_param", (ctypes.c_double * 4) * 4),
        ("reg", ctypes.c_int),
        ("scheme", ctypes.c_int),
        ("nz", ctypes.c_int),
        ("z0", ctypes.c_double), ("z1", ctypes.c_double),
        ("bc_z", ctypes.c_int * 2),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("faces", ctypes.c_longlong), ("iters_total", ctypes.c_longlong),
        ("iters_max", ctypes.c_int), ("nonconverged", ctypes.c_longlong),
        ("departure_out", ctypes.c_longlong), ("nonphysical", ctypes.c_longlong),
        ("dt", ctypes.c_double),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(LIB_PATH)
    lib.orc_lattice.restype = ctypes.c_int
    lib.orc_lattice.argtypes = [ctypes.c_int, _D, _D]
    lib.orc_moments.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double, _D]
    lib.orc_grad_project.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double, _D]
    lib.orc_grad_coefficients.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double, _D]
    lib.orc_eq_project.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double, _D]
    lib.orc_limiter.restype = ctypes.c_double
    lib.orc_limiter.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
    for name in ("orc_phibar_plus", "orc_face_recover", "orc_update_relax"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_double
        fn.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [ctypes.POINTER(_Config), _D, _D, _D, _D]
    lib.orc_create3.restype = ctypes.c_void_p
    lib.orc_create3.argtypes = [ctypes.POINTER(_Config), _D, _D, _D, _D, _D]
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_step.restype = ctypes.c_int
    lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(_Stats)]
    lib.orc_time.restype = ctypes.c_double
    lib.orc_time.argtypes = [ctypes.c_void_p]
    lib.orc_steps.restype = ctypes.c_longlong
    lib.orc_steps.argtypes = [ctypes.c_void_p]
    lib.orc_nfaces.restype = ctypes.c_longlong
    lib.orc_nfaces.argtypes = [ctypes.c_void_p]
    lib.orc_fields.argtypes = [ctypes.c_void_p, _D, _D, _D, _D]
    lib.orc_conserved.argtypes = [ctypes.c_void_p, _D]
    lib.orc_populations.argtypes = [ctypes.c_void_p, _D, _D, _D]
    lib.orc_reframed.argtypes = [ctypes.c_void_p, _D, _D, _D]
    lib.orc_face_frames.argtypes = [ctypes.c_void_p, _D]
    lib.orc_set_face_frames.argtypes = [ctypes.c_void_p, _D]
    lib.orc_face_moments.argtypes = [ctypes.c_void_p, _D, _D]
    lib.orc_face_iters.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def lattice(dim: int):
    """Nodes c (Q x dim) and weights W (Q) of Table I (D1Q4 / D2Q16)."""
    lib = _load()
    Q = 4 ** dim
    c = np.zeros((Q, dim))
    W = np.zeros(Q)
    lib.orc_lattice(dim, _ptr(c), _ptr(W))
    return c, W


def nmom(dim: int, order: int) -> int:
    return sum(dim ** k for k in range(order + 1))


def moments(dim: int, order: int, f, u, T) -> np.ndarray:
    """Lab-frame moment tensors M_0..M_order, packed [M0, M1, M2, M3] (row-major)."""
    lib = _load()
    f = _f64(f)
    u = _f64(np.atleast_1d(u))
    out = np.zeros(nmom(dim, order))
    lib.orc_moments(dim, order, _ptr(f), _ptr(u), float(T), _ptr(out))
    return out


def grad_project(dim: int, order: int, M, u, T) -> np.ndarray:
    lib = _load()
    M = _f64(M)
    u = _f64(np.atleast_1d(u))
    out = np.zeros(4 ** dim)
    lib.orc_grad_project(dim, order, _ptr(M), _ptr(u), float(T), _ptr(out))
    return out


def grad_coefficients(dim: int, order: int, M, u, T) -> np.ndarray:
    lib = _load()
    M = _f64(M)
    u = _f64(np.atleast_1d(u))
    out = np.zeros(nmom(dim, order))
    lib.orc_grad_coefficients(dim, order, _ptr(M), _ptr(u), float(T), _ptr(out))
    return out


def eq_project(dim, M, u, T):
    """Populations of the alternative regularization of Sec. II.C (moments of order 0..3
    kept, the other moments at equilibrium in the new frame) with lab moments M (packed
    as for grad_project, order 3) in frame {u, T}."""
    lib = _load()
    M = _f64(M)
    u = _f64(np.atleast_1d(u))
    out = np.zeros(4 ** dim)
    lib.orc_eq_project(dim, _ptr(M), _ptr(u), float(T), _ptr(out))
    return out


def limiter(kind: str, a: float, b: float) -> float:
    return _load().orc_limiter(LIMITER[kind], float(a), float(b))


def phibar_plus(ft, feq, eps):
    return _load().orc_phibar_plus(float(ft), float(feq), float(eps))


def face_recover(pb, feq, eps):
    return _load().orc_face_recover(float(pb), float(feq), float(eps))


def update_relax(ft, feq, eps):
    return _load().orc_update_relax(float(ft), float(feq), float(eps))


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    _load().orc_set_num_threads(int(n))


def _make_config(cfg: dict) -> _Config:
    c = _Config()
    c.dim = int(cfg["dim"])
    c.nx = int(cfg["nx"])
    c.ny = int(cfg.get("ny", 1))
    c.nz = int(cfg.get("nz", 1))
    c.z0, c.z1 = float(cfg.get("z0", 0.0)), float(cfg.get("z1", 1.0))
    c.x0, c.x1 = float(cfg.get("x0", 0.0)), float(cfg.get("x1", 1.0))
    c.y0, c.y1 = float(cfg.get("y0", 0.0)), float(cfg.get("y1", 1.0))
    c.gamma = float(cfg["gamma"])
    c.cfl = float(cfg["cfl"])
    c.mu = float(cfg["mu"])
    c.limiter = LIMITER[cfg.get("limiter", "vanleer")]
    c.tol = float(cfg["tol"])
    c.max_iter = int(cfg["max_iter"])
    c.reg = REGULARIZATION[cfg.get("regularization", "grad")]
    c.scheme = SCHEME[cfg.get("scheme", "fv")]
    bc = cfg["bc"]
    for k in range(2):
        c.bc_z[k] = BC_KIND[bc[4 + k]] if len(bc) > 4 else BC_KIND["outflow"]
    for k in range(4):
        c.bc[k] = BC_KIND[bc[k]]
        for q in range(4):
            c.bc_state[k][q] = float(cfg.get("bc_state", [[0.0] * 4] * 4)[k][q])
            c.bc_alt[k][q] = float(cfg.get("bc_alt", [[0.0] * 4] * 4)[k][q])
            c.bc_param[k][q] = float(cfg.get("bc_param", [[0.0] * 4] * 4)[k][q])
    return c


class Sim:
    """One oracle simulation (a 1D tube, a 2D grid or a 3D box)."""

    def __init__(self, cfg: dict, rho, ux, uy, p, uz=None):
        lib = _load()
        self.cfg = dict(cfg)
        self.dim = int(cfg["dim"])
        self.nx = int(cfg["nx"])
        self.ny = int(cfg.get("ny", 1)) if self.dim >= 2 else 1
        self.nz = int(cfg.get("nz", 1)) if self.dim == 3 else 1
        self.n = self.nx * self.ny * self.nz
        self.Q = 4 ** self.dim
        self._c = _make_config(cfg)
        self._rho = _f64(rho).ravel()
        self._ux = _f64(ux).ravel()
        self._uy = _f64(uy if uy is not None else np.zeros(self.n)).ravel()
        self._uz = _f64(uz if uz is not None else np.zeros(self.n)).ravel()
        self._p = _f64(p).ravel()
        for a in (self._rho, self._ux, self._uy, self._uz, self._p):
            if a.size != self.n:
                raise ValueError("initial field size does not match the grid")
        h = lib.orc_create3(ctypes.byref(self._c), _ptr(self._rho), _ptr(self._ux),
                            _ptr(self._uy), _ptr(self._uz), _ptr(self._p))
        if not h:
            raise ValueError("oracle rejected the configuration or initial state")
        self._h = h
        self.nfaces = lib.orc_nfaces(h)
        self.last = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
        self._h = None

    def step(self, t_end: float = float("inf")) -> int:
        st = _Stats()
        rc = _load().orc_step(self._h, float(t_end), ctypes.byref(st))
        self.last = {k: getattr(st, k) for k, _ in _Stats._fields_}
        return rc

    def run(self, nsteps: int, t_end: float = float("inf")) -> dict:
        agg = {"steps": 0, "iters_total": 0, "faces": 0, "nonconverged": 0, "iters_max": 0}
        for _ in range(nsteps):
            rc = self.step(t_end)
            if rc == 1:
                break
            agg["steps"] += 1
            agg["iters_total"] += self.last["iters_total"]
            agg["faces"] += self.last["faces"]
            agg["nonconverged"] += self.last["nonconverged"]
            agg["iters_max"] = max(agg["iters_max"], self.last["iters_max"])
        return agg

    @property
    def t(self) -> float:
        return _load().orc_time(self._h)

    @property
    def steps(self) -> int:
        return _load().orc_steps(self._h)

    def fields(self):
        """rho, ux, uy (None in 1D), T; in 3D use conserved() for the z momentum."""
        r = np.zeros(self.n); ux = np.zeros(self.n); uy = np.zeros(self.n); T = np.zeros(self.n)
        _load().orc_fields(self._h, _ptr(r), _ptr(ux), _ptr(uy), _ptr(T))
        return r, ux, (uy if self.dim >= 2 else None), T

    def conserved(self) -> np.ndarray:
        U = np.zeros((self.dim + 2, self.n))
        _load().orc_conserved(self._h, _ptr(U))
        return U

    def populations(self):
        f = np.zeros((self.Q, self.n)); g = np.zeros((self.Q, self.n))
        fr = np.zeros((self.dim + 1, self.n))
        _load().orc_populations(self._h, _ptr(f), _ptr(g), _ptr(fr))
        return f, g, fr

    def reframed(self):
        f = np.zeros((self.Q, self.n)); g = np.zeros((self.Q, self.n))
        fr = np.zeros((self.dim + 1, self.n))
        _load().orc_reframed(self._h, _ptr(f), _ptr(g), _ptr(fr))
        return f, g, fr

    def face_frames(self) -> np.ndarray:
        out = np.zeros((self.nfaces, self.dim + 1))
        _load().orc_face_frames(self._h, _ptr(out))
        return out

    def set_face_frames(self, frames) -> None:
        a = _f64(frames).reshape(self.nfaces, self.dim + 1)
        _load().orc_set_face_frames(self._h, _ptr(a))

    def face_moments(self):
        nf3 = nmom(self.dim, 3); ng2 = nmom(self.dim, 2)
        Mf = np.zeros((self.nfaces, nf3)); Mg = np.zeros((self.nfaces, ng2))
        _load().orc_face_moments(self._h, _ptr(Mf), _ptr(Mg))
        return Mf, Mg

    def face_iters(self) -> np.ndarray:
        out = np.zeros(self.nfaces, dtype=np.int32)
        _load().orc_face_iters(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        return out
