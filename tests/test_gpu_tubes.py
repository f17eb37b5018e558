"""GPU parity of the batched 1D shock tubes: many independent tubes of uneven length in one
launch per kernel, each with its own time step and clock, against the FP64 oracle run tube
by tube (FP64 form: relative max-norm error <= 1e-12 per conserved field).

The random tubes reach density ratios of 1e5 and Mach 5 on the light side; under this
build's readings some of them produce a cell with T <= 0 within a few steps, in the oracle
as in the GPU path. Such a tube is frozen on the GPU (the others go on); the tests check
that exactly the tubes that fail in the oracle are flagged, and compare the others."""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu


def _oracle_tube(orc, batch, fields, k, steps, tol=None):
    c = W.tube_config(batch, k)
    if tol is not None:
        c["tol"] = tol
    ff = W.tube_fields(batch, fields, k)
    o = orc.Sim(c, ff["rho"], ff["ux"], None, ff["p"])
    for s in range(steps):
        o.step()
        r, _, _, T = o.fields()
        if not (np.all(np.isfinite(r)) and np.all(np.isfinite(T)) and r.min() > 0 and T.min() > 0):
            return o, s
    return o, None


def _compare(orc, batch, fields, g, steps):
    U, t, failed = g.conserved(), g.time(), g.failed_instances()
    errs, nfail = [], 0
    for k in range(len(batch["lengths"])):
        o, fs = _oracle_tube(orc, batch, fields, k, steps)
        assert bool(failed[k]) == (fs is not None), (k, fs)
        if fs is not None:
            nfail += 1
            continue
        sl = slice(int(batch["offsets"][k]), int(batch["offsets"][k + 1]))
        Uo = o.conserved()
        e = 0.0
        for q in range(3):
            scale = np.abs(Uo[q]).max()
            e = max(e, np.abs(U[q, sl] - Uo[q]).max() / (scale if scale > 0 else 1.0))
        errs.append(e)
        assert t[k] == pytest.approx(o.t, rel=1e-12)
    return np.array(errs), nfail


def test_tube_batch_fp64_parity(orc):
    """Moderate random tubes (density and pressure ratios up to 100, |Mach| <= 2), uneven
    lengths 20..300: the same tubes fail as in the oracle (a cold dense gas hit by a hot
    light one, temperature ratio ~1e3), every other tube within 1e-12 of the oracle."""
    from paper_2203_05477_amd import pond

    batch, fields = W.tube_batch(n_tubes=48, len_lo=20, len_hi=300, tol=1e-13, rho_decades=2.0,
                                 p_decades=2.0, mach=2.0)
    print("case tubes", len(batch["lengths"]), int(batch["lengths"].sum()), flush=True)
    g = pond.Context(batch, fields, precision="fp64")
    g.step(25, check=False)
    errs, nfail = _compare(orc, batch, fields, g, 25)
    print("moderate tubes fp64 err", errs.max(), "failed", nfail, flush=True)
    assert len(errs) >= 30 and errs.max() <= 1e-12


EPS64 = 2.0 ** -52


def _speed_range(batch, k):
    """Largest lab-frame particle speed of tube k's initial states over the smallest thermal
    speed sqrt(T) among them: the conditioning of a transform between the frames of its
    cells, written with lab-frame moments (the oracle's form), is about this number cubed
    (a third-order coefficient is a difference of terms of size rho |u|^3 that leaves
    rho T^(3/2))."""
    (rl, ul, pl), (rr, ur, pr) = batch["states"][k]
    Tl, Tr = pl / rl, pr / rr
    vmax = max(abs(ul) + 2.3344 * np.sqrt(Tl), abs(ur) + 2.3344 * np.sqrt(Tr))
    return vmax / np.sqrt(min(Tl, Tr))


def test_tube_batch_extreme_fp64(orc):
    """The full ranges of the batch generator (density ratio to 1e5, pressure ratio to 1e6,
    |Mach| <= 5), FP64 at iteration tolerance 1e-10 on both sides: the tubes that fail in
    the oracle are exactly the frozen ones, and every other tube k agrees within its own bar
    1e-12 + n (eps M_k^3 + 0.4 tol) after n steps, where M_k is its speed range (above):
    eps M_k^3 is the rounding the oracle's lab-frame algebra leaves per step at that
    conditioning (the kernels' frame-relative algebra is well conditioned), and 0.4 tol per
    step is what two iterations stopped within tol of each other move a cell at CFL 0.2."""
    from paper_2203_05477_amd import pond

    tol, n = 1e-10, 25
    batch, fields = W.tube_batch(n_tubes=48, len_lo=20, len_hi=300, tol=tol)
    g = pond.Context(batch, fields, precision="fp64")
    g.step(n, check=False)
    U, t, failed = g.conserved(), g.time(), g.failed_instances()
    ratios, nfail = [], 0
    for k in range(len(batch["lengths"])):
        o, fs = _oracle_tube(orc, batch, fields, k, n)
        assert bool(failed[k]) == (fs is not None), (k, fs)
        if fs is not None:
            nfail += 1
            continue
        sl = slice(int(batch["offsets"][k]), int(batch["offsets"][k + 1]))
        Uo = o.conserved()
        e = max(np.abs(U[q, sl] - Uo[q]).max() / max(np.abs(Uo[q]).max(), 1e-300) for q in range(3))
        M = _speed_range(batch, k)
        bar = 1e-12 + n * (EPS64 * M ** 3 + 0.4 * tol)
        ratios.append((e / bar, e, M))
        assert t[k] == pytest.approx(o.t, rel=1e-12)
    r = np.array(ratios)
    print("extreme tubes fp64: compared", len(r), "failed", nfail, "max err/bar", r[:, 0].max(),
          "max err", r[:, 1].max(), "speed ranges", np.round(np.sort(r[:, 2]), 1), flush=True)
    assert len(r) >= 5 and np.all(r[:, 0] <= 1.0)


def test_tube_batch_full_size_sampled(orc):
    """The full batch (4096 tubes of 200..4000 cells, seed 220305477) in the launch shape the
    autotuner picks, mixed precision at iteration tolerance 1e-5; sampled tubes against the
    FP64 oracle at the same tolerance: the same tubes fail, and every other sampled tube is
    within relative L1 1e-4 per conserved field and its clock within 1e-6."""
    from paper_2203_05477_amd import pond

    batch, fields = W.tube_batch()
    g = pond.Context(batch, fields, precision="mixed")
    g.autotune()
    st = g.step(16, check=False)
    print("full batch", st["cell_updates"], st["iters_total"] / st["faces"], "failed",
          st["failed_instances"], flush=True)
    U, t, failed = g.conserved(), g.time(), g.failed_instances()
    errs, terr, mism = [], [], []
    for k in list(range(0, 4096, 128)) + [4095]:
        o, fs = _oracle_tube(orc, batch, fields, k, 16)
        if (fs is not None) != bool(failed[k]):
            mism.append(k)
            continue
        if fs is not None:
            continue
        sl = slice(int(batch["offsets"][k]), int(batch["offsets"][k + 1]))
        Uo = o.conserved()
        errs.append(max(np.abs(U[q, sl] - Uo[q]).sum() / max(np.abs(Uo[q]).sum(), 1e-300) for q in range(3)))
        terr.append(abs(t[k] - o.t) / o.t)
    errs, terr = np.array(errs), np.array(terr)
    print("full batch mixed rel L1 (sampled, healthy tubes)", len(errs), np.median(errs), errs.max(),
          "time", np.median(terr), terr.max(), "failure mismatches", mism, flush=True)
    print("per tube", np.round(np.log10(errs + 1e-300), 1), flush=True)
    assert not mism
    assert len(errs) >= 5 and errs.max() < 1e-4 and terr.max() < 1e-6


def test_tube_tiles_bitwise_identical(orc):
    """Every launch shape gives bitwise-identical FP64 results."""
    from paper_2203_05477_amd import pond

    batch, fields = W.tube_batch(n_tubes=40, len_lo=50, len_hi=400, tol=1e-12)
    outs = []
    for bx in (64, 128, 256):
        g = pond.Context(batch, fields, precision="fp64")
        g.set_tiles(bx, 1, 256)
        g.step(10, check=False)
        outs.append(g.conserved())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
