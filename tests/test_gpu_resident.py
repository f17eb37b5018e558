"""The resident 1D path (pond_set_resident: every step of a pond_step call in one launch,
one block per tube) against the launched kernels: the same bits for the state, the face
frames, the counters and the failure flags, in both precisions."""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu

COUNTERS = ("cell_updates", "converged_cell_updates", "faces", "iters_total", "iters_max",
            "nonconverged", "fallback", "departure_out", "failed_instances")


def _pair(cfg, f, precision):
    from paper_2203_05477_amd import pond

    a = pond.Context(cfg, f, precision=precision)
    b = pond.Context(cfg, f, precision=precision)
    b.set_resident(True)
    return a, b


def _same(a, b):
    assert np.array_equal(a.conserved(), b.conserved(), equal_nan=True)
    fa, ga, ra = a.populations()
    fb, gb, rb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb) and np.array_equal(ra, rb)
    assert np.array_equal(a.face_frames(), b.face_frames(), equal_nan=True)
    assert np.array_equal(a.time(), b.time())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resident_shock_tube_bitwise(precision):
    """400-cell shock tube to t = 0.2 in uneven calls (1, 2, 37, 100, then to the end): the
    resident launch keeps the step parity across calls and clips the last step to t_end."""
    cfg, f = W.shock_tube(400)
    print("case shock_tube resident", precision, flush=True)
    a, b = _pair(cfg, f, precision)
    for n in (1, 2, 37, 100, 600):
        sa = a.step(n, 0.2)
        sb = b.step(n, 0.2)
        for k in COUNTERS:
            assert sa[k] == sb[k], (n, k, sa[k], sb[k])
        _same(a, b)
    assert b.time()[0] == pytest.approx(0.2, abs=1e-15)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resident_tube_batch_bitwise(precision):
    """Moderate random tubes of uneven length (20..300 cells; some fail within the run and
    are frozen): 25 steps in two calls, the same bits and the same failed tubes."""
    batch, fields = W.tube_batch(n_tubes=48, len_lo=20, len_hi=300, tol=1e-13, rho_decades=2.0,
                                 p_decades=2.0, mach=2.0)
    print("case tubes resident", precision, flush=True)
    a, b = _pair(batch, fields, precision)
    for n in (10, 15):
        sa = a.step(n, check=False)
        sb = b.step(n, check=False)
        assert sa["status"] == sb["status"]
        for k in COUNTERS:
            assert sa[k] == sb[k], (n, k, sa[k], sb[k])
    assert np.array_equal(a.failed_instances(), b.failed_instances())
    assert np.array_equal(a.conserved(), b.conserved(), equal_nan=True)
    assert np.array_equal(a.time(), b.time())
    print("failed tubes", int(np.sum(b.failed_instances())), flush=True)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resident_large_batch_bitwise(precision):
    """300 tubes (at least one per compute unit: the 256-thread blocks) of 20..120 cells,
    full ranges of the generator (many fail and are frozen), 30 steps."""
    batch, fields = W.tube_batch(n_tubes=300, len_lo=20, len_hi=120, tol=1e-10)
    print("case large tube batch resident", precision, flush=True)
    a, b = _pair(batch, fields, precision)
    sa = a.step(30, check=False)
    sb = b.step(30, check=False)
    assert sa["status"] == sb["status"]
    for k in COUNTERS:
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    assert np.array_equal(a.failed_instances(), b.failed_instances())
    assert np.array_equal(a.conserved(), b.conserved(), equal_nan=True)
    assert np.array_equal(a.face_frames(), b.face_frames(), equal_nan=True)
    print("failed tubes", int(np.sum(b.failed_instances())), flush=True)
    a.close()
    b.close()


def test_resident_le_blanc_and_minmod_bitwise():
    """A strong case with first-order fallback faces in most steps (Le Blanc, 4,000 cells,
    four chunks of 1,024 faces per step in mixed precision), and the minmod kernel."""
    from paper_2203_05477_amd import pond

    cfg, f = W.riemann_case("le_blanc", tol=W.TOL_FP32)
    print("case le_blanc resident mixed", flush=True)
    a, b = _pair(cfg, f, "mixed")
    sa, sb = a.step(500, cfg["t_end"]), b.step(500, cfg["t_end"])
    assert sb["fallback"] > 0
    for k in COUNTERS:
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    _same(a, b)
    a.close()
    b.close()
    cfg, f = W.shock_tube(300)
    cfg["limiter"] = "minmod"
    print("case shock_tube minmod resident fp64", flush=True)
    a, b = _pair(cfg, f, "fp64")
    a.step(200, 0.2)
    b.step(200, 0.2)
    _same(a, b)
    a.close()
    b.close()
    cfg, f = W.double_mach(16, 8)
    g = pond.Context(cfg, f, precision="fp64")
    with pytest.raises(pond.PondError):
        g.set_resident(True)
    g.close()
