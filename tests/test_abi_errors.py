"""Error behaviour of the C ABI that the host decides before touching a device (runs on
machines without a GPU): invalid configurations and fields give POND_EINVAL, null handles
are rejected, and a valid configuration without a usable device gives POND_EDEVICE rather
than any fallback."""
import ctypes

import numpy as np
import pytest

from paper_2203_05477_amd import pond
from paper_2203_05477_amd import workloads as W

EINVAL, EDEVICE = 1, 3


def _init_status(cfg, f, precision="fp64"):
    lib = pond.load()
    c, keep = pond.make_config(cfg, precision=precision)
    h = ctypes.c_void_p()
    arrs = [np.ascontiguousarray(np.asarray(f[k], dtype=np.float64)) if f.get(k) is not None else None
            for k in ("rho", "ux", "uy", "p")]
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None
    st = lib.pond_init(ctypes.byref(c), ptr(arrs[0]), ptr(arrs[1]), ptr(arrs[2]), ptr(arrs[3]), ctypes.byref(h))
    if st == 0:
        lib.pond_free(h)
    else:
        assert not h.value  # *out = NULL on error
    del keep
    return st


def _cases():
    out = []

    def add(name, mutate_cfg=None, mutate_f=None, base="tube"):
        cfg, f = W.shock_tube(32) if base == "tube" else W.double_mach(16, 8)
        f = {k: (None if v is None else np.array(v, dtype=np.float64)) for k, v in f.items()}
        if mutate_cfg:
            mutate_cfg(cfg)
        if mutate_f:
            mutate_f(f)
        out.append(pytest.param(cfg, f, id=name))

    add("gamma_le_1", lambda c: c.update(gamma=1.0))
    add("gamma_cv_too_small_2d", lambda c: c.update(gamma=2.5), base="dmr")
    add("cfl_ge_1", lambda c: c.update(cfl=1.0))
    add("cfl_zero", lambda c: c.update(cfl=0.0))
    add("mu_zero", lambda c: c.update(mu=0.0))
    add("tol_zero", lambda c: c.update(tol=0.0))
    add("max_iter_zero", lambda c: c.update(max_iter=0))
    add("empty_domain", lambda c: c.update(x1=c["x0"]))
    add("too_few_cells_1d", lambda c: c.update(nx=3), lambda f: f.update({k: f[k][:3] for k in ("rho", "ux", "p")}))
    add("negative_density", None, lambda f: f["rho"].__setitem__(5, -1.0))
    add("zero_pressure", None, lambda f: f["p"].__setitem__(0, 0.0))
    add("nan_velocity", None, lambda f: f["ux"].__setitem__(7, np.nan))
    add("unpaired_periodic", lambda c: c["bc"].__setitem__(0, "periodic"))
    add("fixed_side_without_state", lambda c: c["bc"].__setitem__(0, "fixed"))
    add("too_few_cells_2d", lambda c: c.update(ny=1), lambda f: f.update({k: f[k][:16] for k in ("rho", "ux", "uy", "p")}), base="dmr")
    add("missing_uy_2d", None, lambda f: f.update(uy=None), base="dmr")
    add("nan_uy_2d", None, lambda f: f["uy"].__setitem__(3, np.nan), base="dmr")
    return out


@pytest.mark.parametrize("cfg,f", _cases())
def test_invalid_input_is_rejected(cfg, f):
    assert _init_status(cfg, f) == EINVAL


def test_unknown_flag_bits_are_rejected():
    """Only POND_FLAG_STRICT, POND_FLAG_REG_EQ and POND_FLAG_SEMI_LAGRANGIAN are defined:
    any other bit is an error."""
    lib = pond.load()
    cfg, f = W.double_mach(16, 8)
    c, keep = pond.make_config(cfg)
    c.flags = 8
    arrs = [np.ascontiguousarray(np.asarray(f[k], dtype=np.float64)) for k in ("rho", "ux", "uy", "p")]
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    assert lib.pond_init(ctypes.byref(c), *[P(a) for a in arrs], ctypes.byref(h)) == EINVAL
    assert not h.value
    c2, _ = pond.make_config(dict(cfg, regularization="eq"))
    assert c2.flags == pond.FLAG_REG_EQ


def test_batch_rules():
    """A batch needs tubes of at least 4 cells and no periodic ends."""
    cfg, f = W.tube_batch(n_tubes=3, len_lo=10, len_hi=20)
    cfg["lengths"] = np.array([10, 3, 12], dtype=np.int32)
    n = int(cfg["lengths"].sum())
    g = {"rho": np.ones(n), "ux": np.zeros(n), "uy": None, "p": np.ones(n)}
    assert _init_status(cfg, g) == EINVAL
    cfg, f = W.tube_batch(n_tubes=3, len_lo=10, len_hi=20)
    cfg["bc"] = ["periodic", "periodic", "outflow", "outflow"]
    assert _init_status(cfg, f) == EINVAL


def test_valid_input_without_device_fails_loudly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present: the valid configuration would run")
    cfg, f = W.shock_tube(32)
    assert _init_status(cfg, f) == EDEVICE
    with pytest.raises(pond.PondError):
        pond.Context(cfg, f)


def test_null_handles_and_strerror():
    lib = pond.load()
    P = ctypes.c_void_p
    assert lib.pond_step(P(), 1, 1.0, None) == EINVAL
    assert lib.pond_set_iter_split(P(), 2) == EINVAL
    assert lib.pond_set_graph(P(), 1) == EINVAL
    assert lib.pond_set_resident(P(), 1) == EINVAL
    assert lib.pond_set_tiles(P(), 8, 8, 256) == EINVAL
    assert lib.pond_autotune(P()) == EINVAL
    assert lib.pond_kernel_times(P(), None) == EINVAL
    assert lib.pond_nfaces(P()) == 0
    assert lib.pond_save(P(), b"/tmp/x.ckpt") == EINVAL
    assert lib.pond_load(P(), b"/tmp/x.ckpt") == EINVAL
    lib.pond_free(P())  # no-op
    names = [lib.pond_strerror(s).decode() for s in range(8)]
    assert names[0] == "ok" and len(set(names)) == 8
    assert lib.pond_strerror(99) == b"unknown status"


def test_semi_lagrangian_is_refused_in_3d():
    """The semi-Lagrangian step is built in 1D and 2D: pond_init3 refuses the flag."""
    lib = pond.load()
    cfg, f = W.random_smooth_3d(6, 5, 4, seed=1)
    c, keep = pond.make_config(dict(cfg, scheme="sl"))
    assert c.flags & pond.FLAG_SEMI_LAGRANGIAN
    arrs = [np.ascontiguousarray(np.asarray(f[k], dtype=np.float64)) for k in ("rho", "ux", "uy", "uz", "p")]
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    assert lib.pond_init3(ctypes.byref(c), *[P(a) for a in arrs], ctypes.byref(h)) == EINVAL
    assert not h.value
    del keep
