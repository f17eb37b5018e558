"""GPU parity at the full sizes of the 2D workloads, in the launch configuration the
benchmark times (autotuned face tiles, default hand-over to the tail kernel), for the first
steps, against the FP64 oracle run on the host's cores.

FP64: element-wise to 1e-12 while every face ends its iteration the same way on both sides;
a face whose iteration sits at the iteration cap may end differently under another
rounding order, and then only the cells next to it may differ (the comparison stops
there). Mixed precision: relative L1 distance to the oracle below 1e-4 per conserved field.
"""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _face_cells(cfg, faces):
    nx = cfg["nx"]
    nfx = (nx + 1) * cfg["ny"]
    cells = set()
    for k in faces:
        if k < nfx:
            i, j = k % (nx + 1), k // (nx + 1)
            cells.update({(j, i - 1), (j, i)})
        else:
            i, j = (k - nfx) % nx, (k - nfx) // nx
            cells.update({(j - 1, i), (j, i)})
    return cells


def _bench_context(cfg, f, precision):
    from paper_2203_05477_amd import pond

    g = pond.Context(cfg, f, precision=precision)
    g.autotune()
    return g


def _oracle(orc, cfg, f):
    return orc.Sim(cfg, f["rho"], f["ux"], f["uy"], f["p"])


def _lockstep_fp64(orc, cfg, f, steps, name):
    g = _bench_context(cfg, f, "fp64")
    o = _oracle(orc, cfg, f)
    nx, ny = cfg["nx"], cfg["ny"]
    compared = 0
    for k in range(steps):
        o.step()
        g.step(1)
        assert g.time()[0] == pytest.approx(o.t, rel=1e-14)
        Ug, Uo = g.conserved(), o.conserved()
        scale = np.abs(Uo).max(axis=1, keepdims=True)
        scale[1:-1] = np.abs(Uo[1:-1]).max()
        d = (np.abs(Ug - Uo) / scale).max(axis=0).reshape(ny, nx)
        split = np.nonzero((g.face_iters() > 0) != (o.face_iters() > 0))[0]
        print(name, "step", k, "max rel err", d.max(), "split faces", len(split), flush=True)
        if len(split) == 0:
            assert d.max() <= TOL64, (k, d.max())
            compared += 1
            continue
        off = {tuple(c) for c in np.argwhere(d > TOL64)}
        assert off <= _face_cells(cfg, split), (k, sorted(off - _face_cells(cfg, split))[:5])
        break
    return compared


def test_double_mach_full_size_fp64(orc):
    """1920 x 480 double Mach reflection, first 3 steps."""
    cfg, f = W.double_mach(1920, 480)
    print("case dmr 1920x480 fp64", flush=True)
    assert _lockstep_fp64(orc, cfg, f, 3, "dmr") >= 1


def test_double_mach_full_size_fp64_100_steps(orc):
    """1920 x 480 double Mach reflection, 100 steps in the benchmark's launch configuration,
    GPU FP64 against the oracle, both at tol 1e-13. Past the first faces whose iteration
    ends differently on the two sides (a face at the iteration cap, or a two-cycle stop
    decided within rounding of its threshold, takes the fallback on one side only), the
    cells behind such faces differ at O(1) and their neighbours follow; everything else
    stays at rounding. Bars: at least 99% of the cells within 1e-12 of the oracle, the
    clocks within 1e-12, and the relative L1 distance of every conserved field below 1e-4."""
    cfg, f = W.double_mach(1920, 480)
    print("case dmr 1920x480 fp64 100 steps", flush=True)
    g = _bench_context(cfg, f, "fp64")
    o = _oracle(orc, cfg, f)
    for k in range(100):
        o.step()
        g.step(1)
        if k % 20 == 19:
            print("  step", k + 1, flush=True)
    assert g.time()[0] == pytest.approx(o.t, rel=1e-12)
    Ug, Uo = g.conserved(), o.conserved()
    scale = np.abs(Uo).max(axis=1, keepdims=True)
    scale[1:-1] = np.abs(Uo[1:-1]).max()
    d = (np.abs(Ug - Uo) / scale).max(axis=0)
    good = float(np.mean(d <= TOL64))
    l1 = np.abs(Ug - Uo).sum(axis=1) / np.abs(Uo).sum(axis=1)
    print("dmr 100 steps: cells within 1e-12", int((d <= TOL64).sum()), "of", d.size,
          "rel L1", l1, flush=True)
    assert good >= 0.99
    assert np.all(l1 < 1e-4)


def test_shocked_interface_full_size_fp64(orc):
    """2048 x 512 shocked interface, first 3 steps."""
    cfg, f = W.shocked_interface(tol=1e-13)
    print("case shocked interface 2048x512 fp64", flush=True)
    assert _lockstep_fp64(orc, cfg, f, 3, "shocked_interface") >= 1


def test_jet_full_size_fp64(orc):
    """2048 x 2048 Mach-80 jet. Encodes a KNOWN DEPARTURE from Sec. IV.C.5, where the paper
    runs the jet (on [1000,500] cells); under the readings adopted here it loses positivity (the
    oracle's expected-failure test asserts the paper's outcome on a small grid). Tested here:
    the first step element-wise; in the second, the front of the jet one cell inside the
    inflow boundary reaches T < 0, in the oracle as on the GPU, and the same cells fail on
    both sides (failure detection parity)."""
    cfg, f = W.jet(tol=1e-13)
    print("case jet 2048x2048 fp64", flush=True)
    g = _bench_context(cfg, f, "fp64")
    o = _oracle(orc, cfg, f)
    o.step()
    g.step(1)
    Ug, Uo = g.conserved(), o.conserved()
    scale = np.abs(Uo).max(axis=1, keepdims=True)
    scale[1:-1] = np.abs(Uo[1:-1]).max()
    err = (np.abs(Ug - Uo) / scale).max()
    print("jet step 0 max rel err", err, flush=True)
    assert err <= TOL64
    o.step()
    st = g.step(1, check=False)
    To = o.fields()[3]
    Tg = g.moments()[3]
    bad_o = set(np.nonzero(~(To > 0))[0].tolist())
    bad_g = set(np.nonzero(~(Tg > 0))[0].tolist())
    print("jet step 1 non-physical cells: oracle", len(bad_o), "gpu", len(bad_g), "status", st["status"], flush=True)
    assert len(bad_o) > 0 and bad_g == bad_o
    assert st["failed_instances"] == 1


def test_double_mach_full_size_mixed(orc):
    """1920 x 480 double Mach reflection in mixed precision (FP32 iteration tolerance
    1e-5), 5 steps: relative L1 distance to the FP64 oracle (tolerance 1e-10) below 1e-4."""
    cfg, f = W.double_mach(1920, 480, tol=W.TOL_FP32)
    cfo, _ = W.double_mach(1920, 480, tol=W.TOL_FP64)
    print("case dmr 1920x480 mixed", flush=True)
    g = _bench_context(cfg, f, "mixed")
    o = _oracle(orc, cfo, f)
    for _ in range(5):
        o.step()
        g.step(1)
    Ug, Uo = g.conserved(), o.conserved()
    l1 = np.abs(Ug - Uo).sum(axis=1) / np.abs(Uo).sum(axis=1)
    print("dmr mixed rel L1", l1, flush=True)
    assert np.all(l1 < 1e-4)


def test_shocked_interface_full_size_mixed(orc):
    """2048 x 512 shocked interface in mixed precision (FP32 iteration tolerance 1e-5), the
    configuration of the learned frame guess, 5 steps with the plain seed and 5 with the
    seed network (trained on shock-tube and double Mach frames): relative L1 distance to
    the FP64 oracle (tolerance 1e-10) below 1e-4 for both, and the learned form within 1e-5
    of the plain one (the network only moves where an iteration starts; both iterate to the
    same tolerance). The momentum is compared as one vector field: in these first steps the
    transverse momentum is nonzero only around the perturbed interface, at the level of the
    iteration tolerance, so its own relative L1 would measure that tolerance, not an error."""

    def rel(a, b):
        d = np.abs(a - b).sum(axis=1)
        r = np.abs(b).sum(axis=1)
        return np.array([d[0] / r[0], (d[1] + d[2]) / (r[1] + r[2]), d[3] / r[3]])

    from paper_2203_05477_amd import learned_seed as LS
    from paper_2203_05477_amd import pond

    cfg, f = W.shocked_interface(tol=W.TOL_FP32)
    cfo, _ = W.shocked_interface(tol=W.TOL_FP64)
    print("case shocked interface 2048x512 mixed", flush=True)
    o = _oracle(orc, cfo, f)
    for _ in range(5):
        o.step()
    Uo = o.conserved()
    out = {}
    ch, fh = W.double_mach(480, 120, tol=W.TOL_FP32)
    c1, f1 = W.shock_tube(400, tol=W.TOL_FP32)
    cs, fs = W.strip_2d(c1, f1, ny=4)
    data = [LS.harvest(ch, fh, steps=100, precision="mixed", hard_iters=2, every=2),
            LS.harvest(cs, fs, steps=200, precision="mixed", hard_iters=2)]
    net = LS.train(data, epochs=10, batch=4096, lr=2e-3)[0]
    for seed in ("prev", "mlp"):
        g = pond.Context(cfg, f, precision="mixed", seed=seed)
        if seed == "mlp":
            g.load_mlp(net, hard_iters=2)
        g.autotune()
        g.step(5)
        out[seed] = g.conserved()
        g.close()
        l1 = rel(out[seed], Uo)
        print("shocked interface mixed", seed, "rel L1 (rho, momentum, rho E)", l1, flush=True)
        assert np.all(l1 < 1e-4)
    d = rel(out["mlp"], out["prev"])
    print("learned vs plain rel L1", d, flush=True)
    assert np.all(d < 1e-5)


def test_double_mach_2000_steps_mixed_within_the_l1_gate():
    """The whole 2000-step run of the 1920 x 480 double Mach reflection (autotuned tiles, the
    default hand-over to the tail kernel): the mixed form against the FP64 form at the same
    iteration tolerance (1e-5), relative L1 of every conserved field below 1e-4 at the end;
    the two clocks agree to 1e-4 (each dt follows the largest CFL rate of the grid, which
    the forms' differences move at that level: 8e-5 after the 2000 steps) and more than
    99.9% of the cell-updates of both runs converged."""
    from paper_2203_05477_amd import pond

    out = {}
    for prec in ("mixed", "fp64"):
        cfg, f = W.double_mach(1920, 480, tol=W.TOL_FP32)
        g = pond.Context(cfg, f, precision=prec)
        g.autotune()
        st = g.step(2000, check=False)
        out[prec] = (g.conserved(), g.time()[0], st)
        g.close()
        print("dmr 2000 steps", prec, "t", out[prec][1], "converged share",
              st["converged_cell_updates"] / st["cell_updates"], flush=True)
        assert st["status"] == 0 and st["converged_cell_updates"] > 0.999 * st["cell_updates"]
    (Um, tm, _), (Ud, td, _) = out["mixed"], out["fp64"]
    l1 = np.abs(Um - Ud).sum(axis=1) / np.abs(Ud).sum(axis=1)
    print("dmr 2000 steps mixed vs fp64 same tol, rel L1", l1, flush=True)
    assert tm == pytest.approx(td, rel=1e-4)
    assert np.all(l1 < 1e-4)
