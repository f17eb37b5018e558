"""GPU parity on the further 1D Riemann problems the paper prints (Lax, strong shock tube,
Le Blanc, 1D jet; double rarefaction): the FP64 HIP path against the FP64 oracle step by
step, and the mixed form against the exact solution."""
import numpy as np
import pytest

import exact_riemann as ER
from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = ("lax", "strong_shock", "le_blanc", "jet_1d")
TOL64 = 1e-12

# Iteration tolerance of the parity runs: 1e-13 as in the other parity tests, except for
# the Mach-80 jet, where |u|/sqrt(T) ~ 100 puts the rounding floor of the frame change
# near 1e-12: at 1e-12 or 1e-11 faces of the uniform jet stop on 2-cycles of rounding
# noise, and whether a face near the front does so differs between the two sides. The
# jet therefore runs at the FP64 form's production tolerance. Its shock front stops about
# one face per step on a 2-cycle, detected by comparing two FP64 frame distances; a few
# hundred steps in, one such comparison lands within rounding of its threshold and the two
# sides take different, equally valid branches (the measured run diverges at step ~850).
# Its element-wise parity is checked over the first 500 steps; the full run is compared
# through its error against the exact solution.
PARITY_TOL = {"lax": 1e-13, "strong_shock": 1e-13, "le_blanc": 1e-13, "jet_1d": 1e-10}
PARITY_STEPS = {"jet_1d": 500}


def _bar(name, n):
    """Parity bar after n steps. Each side stops a face's iteration once the frame change
    is below tol, so the two final frames of a face can differ by up to ~2 tol; at
    CFL 0.2 that moves a cell's conserved variables by at most ~0.4 tol of their scale
    per step, accumulated over n steps. Le Blanc adds the conditioning of the oracle's
    projection, which takes lab-frame moments as the paper writes them: in the cold gas
    behind the front (T ~ 1e-7, |u| ~ 0.3) their subtraction loses |u|^2/T ~ 1e6 of the
    16 digits, i.e. ~1e-10 of the field scale."""
    return 1e-12 + 0.4 * n * PARITY_TOL[name] + (1e-10 if name == "le_blanc" else 0.0)


def _relerr(a, b):
    return np.array([np.abs(a[k] - b[k]).max() / max(np.abs(b[k]).max(), 1e-300)
                     for k in range(b.shape[0])])


def _l1_exact(name, nx, t, U):
    left, right, xi, (a, b), g = W.RIEMANN_CASES[name][:5]
    ex = ER.cell_average(left, right, g, np.linspace(a, b, nx + 1), xi, t)
    return np.array([np.abs(U[k] - ex[k]).sum() / np.abs(ex[k]).sum() for k in range(3)])


@pytest.mark.parametrize("name", CASES)
def test_riemann_problem_fp64_parity(orc, name):
    """400 cells to the printed final time (2,000-3,200 steps, first-order fallback faces
    at the strong fronts in most steps): conserved fields within the bar above of the
    oracle after every 50th step and at the end, the same final time, and the face frames
    the next step would start from (the jet: over its first 500 steps, then the same error
    against the exact solution at the end, to 1%)."""
    from paper_2203_05477_amd import pond

    cfg, f = W.riemann_case(name, nx=400, tol=PARITY_TOL[name])
    print("case", name, "nx", 400, flush=True)
    g = pond.Context(cfg, f, precision="fp64")
    o = orc.Sim(cfg, f["rho"], f["ux"], None, f["p"])
    t_end = cfg["t_end"]
    last = PARITY_STEPS.get(name)
    n = 0
    while o.t < t_end * (1 - 1e-12):
        o.step(t_end)
        g.step(1, t_end)
        n += 1
        if n % 50 == 0 and (last is None or n <= last):
            e = _relerr(g.conserved(), o.conserved())
            assert e.max() <= _bar(name, n), (name, n, e)
        if n == last:
            ff, fo = g.face_frames(), o.face_frames()
            assert np.abs(ff - fo).max() <= _bar(name, n) * np.abs(fo).max()
    assert g.time()[0] == pytest.approx(o.t, rel=1e-13)
    if last is not None:
        eg = _l1_exact(name, 400, o.t, g.conserved())
        eo = _l1_exact(name, 400, o.t, o.conserved())
        print(name, "steps", n, "L1 gpu", eg, "oracle", eo, flush=True)
        assert np.all(np.abs(eg - eo) <= 0.01 * eo)
        g.close()
        return
    e = _relerr(g.conserved(), o.conserved())
    ff, fo = g.face_frames(), o.face_frames()
    ef = np.abs(ff - fo).max() / np.abs(fo).max()
    print(name, "steps", n, "err", e.max(), "frames", ef, "bar", _bar(name, n), flush=True)
    assert e.max() <= _bar(name, n)
    assert ef <= _bar(name, n)
    g.close()


@pytest.mark.parametrize("name", CASES)
def test_riemann_problem_mixed_error_matches_fp64(orc, name):
    """At the paper's resolution (600 to 4,000 cells), the mixed form (FP32 populations,
    FP64 conserved variables, tol 1e-5) is no less accurate than the FP64 form (tol 1e-10):
    its L1 error against the exact solution is at most 1% above the FP64 form's in every
    conserved field (the strong shock tube's is lower: fewer of its faces stop on a 2-cycle
    at the looser tolerance and fall back to the first-order state)."""
    from paper_2203_05477_amd import pond

    errs = {}
    for prec, tol in (("mixed", W.TOL_FP32), ("fp64", W.TOL_FP64)):
        cfg, f = W.riemann_case(name, tol=tol)
        print("case", name, prec, cfg["nx"], flush=True)
        g = pond.Context(cfg, f, precision=prec)
        for _ in range(100):
            st = g.step(1000, cfg["t_end"])
            if st["t_min"] >= cfg["t_end"]:
                break
        assert g.time()[0] == pytest.approx(cfg["t_end"], rel=1e-13)
        errs[prec] = _l1_exact(name, cfg["nx"], g.time()[0], g.conserved())
        g.close()
    print(name, "L1 mixed", errs["mixed"], "fp64", errs["fp64"], flush=True)
    assert np.all(errs["mixed"] <= 1.01 * errs["fp64"])


def test_double_rarefaction_failure_detected_in_the_same_step(orc):
    """Encodes a KNOWN DEPARTURE from Sec. IV.B (the paper runs this case to t = 0.1; under
    the readings adopted here the step loses positivity next to the centre, see the oracle's
    expected-failure test). What is tested here is failure detection parity: the GPU keeps
    parity with the oracle up to the step whose update leaves a cell with T <= 0, reports
    POND_ENONPHYS for that very step and freezes the tube."""
    from paper_2203_05477_amd import pond

    cfg, f = W.riemann_case("double_rarefaction", nx=800)
    print("case double_rarefaction nx 800", flush=True)
    g = pond.Context(cfg, f, precision="fp64")
    o = orc.Sim(cfg, f["rho"], f["ux"], None, f["p"])
    failed = None
    for n in range(1, 51):
        o.step(cfg["t_end"])
        st = g.step(1, cfg["t_end"], check=False)
        _, _, _, T = o.fields()
        if not (T.min() > 0):
            failed = n
            assert st["status"] == pond.ENONPHYS and st["failed_instances"] == 1
            break
        assert st["status"] == pond.OK, (n, st)
        e = _relerr(g.conserved(), o.conserved())
        assert e.max() <= TOL64, (n, e)
    print("double rarefaction fails at step", failed, flush=True)
    assert failed is not None
    t = g.time()[0]
    st = g.step(1, cfg["t_end"], check=False)
    assert g.time()[0] == t  # frozen
    g.close()


def test_blast_waves_fp64_parity_and_closed_tube(orc):
    """Two blast waves between reflecting ends, 400 cells to t = 0.038 (about 5,300 steps,
    first-order fallback faces at both fronts in most steps): the GPU within the tolerance
    bar of the oracle over the first 1,000 steps (later a stop decision of one of those
    faces lands within rounding of its threshold, as in the jet, and the runs take
    different valid branches), the same final time and density peak to 1%, and mass and
    energy of the closed tube conserved to round-off in both precisions."""
    from paper_2203_05477_amd import pond

    cfg, f = W.blast_waves(400)
    print("case blast_waves 400", flush=True)
    g = pond.Context(cfg, f, precision="fp64")
    o = orc.Sim(cfg, f["rho"], f["ux"], None, f["p"])
    U0 = g.conserved().sum(axis=1)
    n, first_split = 0, None
    while o.t < cfg["t_end"] * (1 - 1e-12):
        o.step(cfg["t_end"])
        g.step(1, cfg["t_end"])
        n += 1
        if n % 100 == 0 and first_split is None:
            e = _relerr(g.conserved(), o.conserved())
            if e.max() > 1e-12 + 0.4 * n * cfg["tol"]:
                first_split = n
    print("blast steps", n, "first step beyond the bar", first_split, flush=True)
    assert first_split is None or first_split > 1000
    assert g.time()[0] == pytest.approx(o.t, rel=1e-13)
    rg, ro = g.moments()[0], o.fields()[0]
    assert rg.max() == pytest.approx(ro.max(), rel=1e-2)
    U1 = g.conserved().sum(axis=1)
    assert abs(U1[0] - U0[0]) <= 1e-12 * U0[0] and abs(U1[2] - U0[2]) <= 1e-12 * U0[2]
    g.close()
    cfgm, _ = W.blast_waves(400, tol=W.TOL_FP32)
    m = pond.Context(cfgm, f, precision="mixed")
    m.step(20000, cfg["t_end"])
    U1 = m.conserved().sum(axis=1)
    assert abs(U1[0] - U0[0]) <= 1e-12 * U0[0] and abs(U1[2] - U0[2]) <= 1e-12 * U0[2]
    m.close()
