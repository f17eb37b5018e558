"""ctypes binding of libpond (include/pond.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libpond.so; this module converts
configuration dicts and numpy arrays to the C ABI and back. There is no fallback: if
the library is missing or no gfx950 device is usable, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpond.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ECFL, ENONPHYS, ESTATE = range(8)
BC = {"periodic": 0, "outflow": 1, "reflect": 2, "fixed": 3, "fixed_window": 4,
      "split_fixed_reflect": 5, "moving_shock": 6}
LIMITER = {"vanleer": 0, "minmod": 1}
PRECISION = {"fp64": 0, "mixed": 1}
SEED = {"prev": 0, "mlp": 1}
FLAG_STRICT = 1
FLAG_REG_EQ = 2
FLAG_SEMI_LAGRANGIAN = 4
LAYOUT = {"hermite": 0, "populations": 1}  # pond_set_state_layout


class PondError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {_strerror(status)} (status {status})")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("n_inst", ctypes.c_int32), ("len", ctypes.POINTER(ctypes.c_int32)),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double),
        ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("mu", ctypes.c_double),
        ("limiter", ctypes.c_int32), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("seed_mode", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 4),
        ("bc_state", (ctypes.c_double * 4) * 4),
        ("bc_alt", (ctypes.c_double * 4) * 4),
        ("bc_param", (ctypes.c_double * 4) * 4),
        ("nz", ctypes.c_int32),
        ("z0", ctypes.c_double), ("z1", ctypes.c_double),
        ("bc_z", ctypes.c_int32 * 2),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("cell_updates", ctypes.c_int64),
        ("converged_cell_updates", ctypes.c_int64), ("faces", ctypes.c_int64),
        ("iters_total", ctypes.c_int64), ("iters_max", ctypes.c_int32),
        ("nonconverged", ctypes.c_int64), ("fallback", ctypes.c_int64),
        ("departure_out", ctypes.c_int64),
        ("t_min", ctypes.c_double), ("t_max", ctypes.c_double),
        ("dt_min", ctypes.c_double), ("dt_max", ctypes.c_double),
        ("failed_instances", ctypes.c_int32),
        ("tail_faces", ctypes.c_int64), ("tail_iters", ctypes.c_int64),
        ("rho_min", ctypes.c_double), ("T_min", ctypes.c_double),
        ("totals", ctypes.c_double * 5),
        ("first_failed_instance", ctypes.c_int32),
        ("first_failed_cell", ctypes.c_int64), ("first_nonconv_face", ctypes.c_int64),
    ]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_}
        out["totals"] = list(self.totals)
        return out


class TrainCfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_P = ctypes.c_void_p


def load(path: str | None = None):
    """Load libpond.so (built in-tree by paper_2203_05477_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime under the same soname as ROCm's: load it first so
    # that torch (device memory, streams) and libpond share one runtime in the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"libpond.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    S = ctypes.c_int
    sig = {
        "pond_init": (S, [ctypes.POINTER(Config), _D, _D, _D, _D, ctypes.POINTER(_P)]),
        "pond_init3": (S, [ctypes.POINTER(Config), _D, _D, _D, _D, _D, ctypes.POINTER(_P)]),
        "pond_step": (S, [_P, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(Stats)]),
        "pond_moments": (S, [_P, _D, _D, _D, _D]),
        "pond_moments_device": (S, [_P, _P]),
        "pond_conserved": (S, [_P, _D]),
        "pond_populations": (S, [_P, _D, _D, _D]),
        "pond_nfaces": (ctypes.c_int64, [_P]),
        "pond_face_frames": (S, [_P, _D]),
        "pond_set_face_frames": (S, [_P, _D]),
        "pond_face_moments": (S, [_P, _D, _D]),
        "pond_face_iters": (S, [_P, ctypes.POINTER(ctypes.c_int32)]),
        "pond_time": (S, [_P, _D]),
        "pond_failed_instances": (S, [_P, ctypes.POINTER(ctypes.c_int32)]),
        "pond_set_stream": (S, [_P, _P]),
        "pond_set_tiles": (S, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
        "pond_get_tiles": (S, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32)]),
        "pond_autotune": (S, [_P]),
        "pond_set_iter_split": (S, [_P, ctypes.c_int32]),
        "pond_set_state_layout": (S, [_P, ctypes.c_int32]),
        "pond_set_graph": (S, [_P, ctypes.c_int32]),
        "pond_set_resident": (S, [_P, ctypes.c_int32]),
        "pond_save": (S, [_P, ctypes.c_char_p]),
        "pond_load": (S, [_P, ctypes.c_char_p]),
        "pond_enable_timing": (S, [_P, ctypes.c_int32]),
        "pond_kernel_times": (S, [_P, _D]),
        "pond_free": (None, [_P]),
        "pond_mlp_nparams": (ctypes.c_int32, []),
        "pond_mlp_create": (S, [ctypes.POINTER(ctypes.c_float), ctypes.c_uint64, ctypes.POINTER(_P)]),
        "pond_mlp_get": (S, [_P, ctypes.POINTER(ctypes.c_float)]),
        "pond_mlp_set": (S, [_P, ctypes.POINTER(ctypes.c_float)]),
        "pond_mlp_forward": (S, [_P, _P, ctypes.c_int64, _P, _P]),
        "pond_mlp_grad": (S, [_P, _P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_float),
                              ctypes.POINTER(ctypes.c_float)]),
        "pond_mlp_train": (S, [_P, _P, _P, ctypes.c_int64, ctypes.POINTER(TrainCfg),
                               ctypes.POINTER(ctypes.c_float)]),
        "pond_mlp_train_noalloc": (S, [_P, _P, _P, ctypes.c_int64, ctypes.POINTER(TrainCfg),
                                       ctypes.POINTER(ctypes.c_float)]),
        "pond_mlp_free": (None, [_P]),
        "pond_mlp_features": (S, [_P, _P, _P]),
        "pond_mlp_targets": (S, [_P, _P, _P, _P]),
        "pond_load_mlp": (S, [_P, _P, ctypes.c_int32]),
        "pond_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "pond_abi_version": (ctypes.c_int32, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names the header declares (checked against the library by the CPU tests)."""
    return ["pond_init", "pond_init3", "pond_step", "pond_moments", "pond_moments_device", "pond_conserved",
            "pond_populations", "pond_nfaces", "pond_face_frames", "pond_set_face_frames",
            "pond_face_moments", "pond_face_iters", "pond_time", "pond_failed_instances",
            "pond_set_stream",
            "pond_set_tiles", "pond_get_tiles", "pond_autotune", "pond_set_iter_split", "pond_set_state_layout",
            "pond_set_graph",
            "pond_set_resident",
            "pond_save", "pond_load",
            "pond_enable_timing",
            "pond_kernel_times", "pond_free", "pond_strerror", "pond_abi_version",
            "pond_mlp_nparams", "pond_mlp_create", "pond_mlp_get", "pond_mlp_set",
            "pond_mlp_forward", "pond_mlp_grad", "pond_mlp_train", "pond_mlp_train_noalloc", "pond_mlp_free",
            "pond_mlp_features", "pond_mlp_targets", "pond_load_mlp"]


def _strerror(s):
    try:
        return load().pond_strerror(int(s)).decode()
    except Exception:  # library not loadable: the status number is still reported
        return "status"


def _ptr(a):
    return a.ctypes.data_as(_D)


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64)).ravel()
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def make_config(cfg: dict, precision="fp64", seed="prev", strict=False) -> tuple[Config, object]:
    c = Config()
    c.dim = int(cfg["dim"])
    lens = cfg.get("lengths")
    keep = None
    if c.dim == 1 and lens is not None:
        keep = np.ascontiguousarray(np.asarray(lens, dtype=np.int32))
        c.n_inst = int(keep.size)
        c.len = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        c.nx = int(keep.sum())
    else:
        c.n_inst = 1
        c.len = None
        c.nx = int(cfg["nx"])
    c.ny = int(cfg.get("ny", 1)) if c.dim >= 2 else 1
    c.nz = int(cfg.get("nz", 1)) if c.dim == 3 else 1
    c.z0, c.z1 = float(cfg.get("z0", 0.0)), float(cfg.get("z1", 1.0))
    c.x0, c.x1 = float(cfg.get("x0", 0.0)), float(cfg.get("x1", 1.0))
    c.y0, c.y1 = float(cfg.get("y0", 0.0)), float(cfg.get("y1", 1.0))
    c.gamma, c.cfl, c.mu = float(cfg["gamma"]), float(cfg["cfl"]), float(cfg["mu"])
    c.limiter = LIMITER[cfg.get("limiter", "vanleer")]
    c.tol = float(cfg["tol"])
    c.max_iter = int(cfg["max_iter"])
    c.precision = PRECISION[precision]
    c.seed_mode = SEED[seed]
    c.flags = ((FLAG_STRICT if strict else 0) | (FLAG_REG_EQ if cfg.get("regularization", "grad") == "eq" else 0)
               | (FLAG_SEMI_LAGRANGIAN if cfg.get("scheme", "fv") == "sl" else 0))
    z = [[0.0] * 4] * 4
    for k in range(2):
        c.bc_z[k] = BC[cfg["bc"][4 + k]] if len(cfg["bc"]) > 4 else BC["outflow"]
    for k in range(4):
        c.bc[k] = BC[cfg["bc"][k]]
        for q in range(4):
            c.bc_state[k][q] = float(cfg.get("bc_state", z)[k][q])
            c.bc_alt[k][q] = float(cfg.get("bc_alt", z)[k][q])
            c.bc_param[k][q] = float(cfg.get("bc_param", z)[k][q])
    return c, keep


class Context:
    """A libpond context: one simulation (a 3D box, a 2D grid, one tube or a batch of tubes)."""

    def __init__(self, cfg: dict, fields: dict, precision="fp64", seed="prev", strict=False):
        lib = load()
        self.cfg = cfg
        self.dim = int(cfg["dim"])
        self._c, self._keep = make_config(cfg, precision, seed, strict)
        self.n = int(self._c.nx) * int(self._c.ny) * int(self._c.nz)
        self.n_inst = int(self._c.n_inst)
        self.Q = 4 ** self.dim
        rho = _f64(fields["rho"], self.n)
        ux = _f64(fields["ux"], self.n)
        uy = _f64(fields["uy"], self.n) if (self.dim >= 2) else None
        uz = _f64(fields["uz"], self.n) if (self.dim == 3) else None
        p = _f64(fields["p"], self.n)
        h = _P()
        st = lib.pond_init3(ctypes.byref(self._c), _ptr(rho), _ptr(ux),
                            _ptr(uy) if uy is not None else None,
                            _ptr(uz) if uz is not None else None, _ptr(p), ctypes.byref(h))
        if st != OK:
            raise PondError(st, "pond_init3")
        self._h = h
        self.nfaces = int(lib.pond_nfaces(h))
        self.last = None

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pond_free(h)
        self._h = None

    __del__ = close

    def step(self, nsteps: int = 1, t_end: float = float("inf"), check=True) -> dict:
        st = Stats()
        rc = load().pond_step(self._h, int(nsteps), float(t_end), ctypes.byref(st))
        self.last = st.as_dict()
        self.last["status"] = rc
        if check and rc != OK:
            raise PondError(rc, "pond_step")
        return self.last

    def moments(self):
        r, ux, uy, T = (np.zeros(self.n) for _ in range(4))
        rc = load().pond_moments(self._h, _ptr(r), _ptr(ux), _ptr(uy), _ptr(T))
        if rc != OK:
            raise PondError(rc, "pond_moments")
        return r, ux, (uy if self.dim >= 2 else None), T

    def moments_device(self, dev_ptr: int):
        rc = load().pond_moments_device(self._h, ctypes.c_void_p(dev_ptr))
        if rc != OK:
            raise PondError(rc, "pond_moments_device")

    def conserved(self):
        U = np.zeros((self.dim + 2, self.n))
        rc = load().pond_conserved(self._h, _ptr(U))
        if rc != OK:
            raise PondError(rc, "pond_conserved")
        return U

    def populations(self):
        f = np.zeros((self.Q, self.n)); g = np.zeros((self.Q, self.n))
        fr = np.zeros((self.dim + 1, self.n))
        rc = load().pond_populations(self._h, _ptr(f), _ptr(g), _ptr(fr))
        if rc != OK:
            raise PondError(rc, "pond_populations")
        return f, g, fr

    def face_frames(self):
        out = np.zeros((self.nfaces, self.dim + 1))
        rc = load().pond_face_frames(self._h, _ptr(out))
        if rc != OK:
            raise PondError(rc, "pond_face_frames")
        return out

    def set_face_frames(self, frames):
        a = _f64(frames, self.nfaces * (self.dim + 1))
        rc = load().pond_set_face_frames(self._h, _ptr(a))
        if rc != OK:
            raise PondError(rc, "pond_set_face_frames")

    def face_moments(self):
        nf3 = sum(self.dim ** k for k in range(4))
        ng2 = sum(self.dim ** k for k in range(3))
        Mf = np.zeros((self.nfaces, nf3)); Mg = np.zeros((self.nfaces, ng2))
        rc = load().pond_face_moments(self._h, _ptr(Mf), _ptr(Mg))
        if rc != OK:
            raise PondError(rc, "pond_face_moments")
        return Mf, Mg

    def face_iters(self):
        out = np.zeros(self.nfaces, dtype=np.int32)
        rc = load().pond_face_iters(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if rc != OK:
            raise PondError(rc, "pond_face_iters")
        return out

    def failed_instances(self):
        out = np.zeros(self.n_inst, dtype=np.int32)
        rc = load().pond_failed_instances(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if rc != OK:
            raise PondError(rc, "pond_failed_instances")
        return out != 0

    def time(self):
        t = np.zeros(self.n_inst)
        rc = load().pond_time(self._h, _ptr(t))
        if rc != OK:
            raise PondError(rc, "pond_time")
        return t

    def set_stream(self, stream_ptr: int | None):
        rc = load().pond_set_stream(self._h, ctypes.c_void_p(stream_ptr or 0))
        if rc != OK:
            raise PondError(rc, "pond_set_stream")

    def set_tiles(self, bx, by, cell_block=256):
        rc = load().pond_set_tiles(self._h, int(bx), int(by), int(cell_block))
        if rc != OK:
            raise PondError(rc, "pond_set_tiles")

    def tiles(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        load().pond_get_tiles(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return a.value, b.value, c.value

    def autotune(self):
        rc = load().pond_autotune(self._h)
        if rc != OK:
            raise PondError(rc, "pond_autotune")
        return self.tiles()

    def enable_timing(self, on=True):
        load().pond_enable_timing(self._h, 1 if on else 0)

    def kernel_times(self):
        """Mean ms per step of each launch of the last step() with timing on: dt, face (the
        face kernel), cell (the cell update kernel; 0 in 2D with a tail kernel), seed, tail
        (2D: the launch that finishes the deferred faces and updates every cell)."""
        out = np.zeros(5)
        load().pond_kernel_times(self._h, _ptr(out))
        return {"dt": out[0], "face": out[1], "cell": out[2], "seed": out[3], "tail": out[4]}

    def save(self, path: str):
        rc = load().pond_save(self._h, str(path).encode())
        if rc != OK:
            raise PondError(rc, "pond_save")

    def load_state(self, path: str):
        rc = load().pond_load(self._h, str(path).encode())
        if rc != OK:
            raise PondError(rc, "pond_load")

    def set_graph(self, on: bool = True):
        rc = load().pond_set_graph(self._h, int(bool(on)))
        if rc != OK:
            raise PondError(rc, "pond_set_graph")

    def set_resident(self, on: bool = True):
        rc = load().pond_set_resident(self._h, int(bool(on)))
        if rc != OK:
            raise PondError(rc, "pond_set_resident")

    def set_iter_split(self, k: int):
        rc = load().pond_set_iter_split(self._h, int(k))
        if rc != OK:
            raise PondError(rc, "pond_set_iter_split")

    def set_state_layout(self, layout: str):
        """"hermite" (the default: 12 Hermite coefficients per 2D cell) or "populations" (the
        32 populations); the current state is converted."""
        rc = load().pond_set_state_layout(self._h, LAYOUT[layout])
        if rc != OK:
            raise PondError(rc, "pond_set_state_layout")


    # ---- learned seed ----
    def mlp_features(self, X_ptr: int, ref_ptr: int):
        rc = load().pond_mlp_features(self._h, ctypes.c_void_p(X_ptr), ctypes.c_void_p(ref_ptr))
        if rc != OK:
            raise PondError(rc, "pond_mlp_features")

    def mlp_targets(self, X_ptr: int, ref_ptr: int, T_ptr: int):
        rc = load().pond_mlp_targets(self._h, ctypes.c_void_p(X_ptr), ctypes.c_void_p(ref_ptr),
                                     ctypes.c_void_p(T_ptr))
        if rc != OK:
            raise PondError(rc, "pond_mlp_targets")

    def load_mlp(self, mlp: "Mlp", hard_iters: int = 2):
        rc = load().pond_load_mlp(self._h, mlp._h, int(hard_iters))
        if rc != OK:
            raise PondError(rc, "pond_load_mlp")


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Mlp:
    """The seed network (BF16 MFMA kernels, FP32 master weights). Device arrays are passed
    as raw device pointers (e.g. torch.Tensor.data_ptr())."""

    def __init__(self, params=None, seed: int = 0):
        lib = load()
        self.nparams = int(lib.pond_mlp_nparams())
        h = _P()
        if params is not None:
            p = np.ascontiguousarray(np.asarray(params, dtype=np.float32)).ravel()
            if p.size != self.nparams:
                raise ValueError("wrong parameter count")
            rc = lib.pond_mlp_create(_fptr(p), ctypes.c_uint64(seed), ctypes.byref(h))
        else:
            rc = lib.pond_mlp_create(None, ctypes.c_uint64(seed), ctypes.byref(h))
        if rc != OK:
            raise PondError(rc, "pond_mlp_create")
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pond_mlp_free(h)
        self._h = None

    __del__ = close

    def params(self):
        p = np.zeros(self.nparams, dtype=np.float32)
        rc = load().pond_mlp_get(self._h, _fptr(p))
        if rc != OK:
            raise PondError(rc, "pond_mlp_get")
        return p

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32)).ravel()
        rc = load().pond_mlp_set(self._h, _fptr(p))
        if rc != OK:
            raise PondError(rc, "pond_mlp_set")

    def forward(self, X_ptr: int, n: int, Y_ptr: int, stream: int | None = None):
        rc = load().pond_mlp_forward(self._h, ctypes.c_void_p(X_ptr), int(n), ctypes.c_void_p(Y_ptr),
                                     ctypes.c_void_p(stream or 0))
        if rc != OK:
            raise PondError(rc, "pond_mlp_forward")

    def grad(self, X_ptr: int, T_ptr: int, n: int):
        g = np.zeros(self.nparams, dtype=np.float32)
        loss = ctypes.c_float()
        rc = load().pond_mlp_grad(self._h, ctypes.c_void_p(X_ptr), ctypes.c_void_p(T_ptr), int(n),
                                  _fptr(g), ctypes.byref(loss))
        if rc != OK:
            raise PondError(rc, "pond_mlp_grad")
        return g, loss.value

    def train(self, X_ptr: int, T_ptr: int, n: int, epochs=10, batch=4096, lr=1e-3,
              beta1=0.9, beta2=0.999, eps=1e-8):
        cfg = TrainCfg(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps))
        out = np.zeros(max(int(epochs), 1), dtype=np.float32)
        rc = load().pond_mlp_train(self._h, ctypes.c_void_p(X_ptr), ctypes.c_void_p(T_ptr), int(n),
                                   ctypes.byref(cfg), _fptr(out))
        if rc != OK:
            raise PondError(rc, "pond_mlp_train")
        return out[: int(epochs)]

    def train_noalloc(self, X_ptr: int, T_ptr: int, n: int, epochs=10, batch=4096, lr=1e-3,
                      beta1=0.9, beta2=0.999, eps=1e-8):
        """pond_mlp_train_noalloc: the same training with the library's static buffers."""
        cfg = TrainCfg(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps))
        out = np.zeros(max(int(epochs), 1), dtype=np.float32)
        rc = load().pond_mlp_train_noalloc(self._h, ctypes.c_void_p(X_ptr), ctypes.c_void_p(T_ptr), int(n),
                                           ctypes.byref(cfg), _fptr(out))
        if rc != OK:
            raise PondError(rc, "pond_mlp_train_noalloc")
        return out[: int(epochs)]
