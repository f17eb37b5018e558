"""Checkpoint and resume (pond_save / pond_load): a run resumed from a file continues
bitwise as the run that wrote it; a file of another configuration is refused and leaves
the context unchanged."""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["dmr_mixed", "dmr_fp64", "tubes_fp64", "dmr_eq_fp64", "tubes_sl_fp64"])
def test_resume_is_bitwise(tmp_path, case):
    from paper_2203_05477_amd import pond

    if case.startswith("dmr"):
        cfg, f = W.double_mach(96, 24, tol=1e-5 if case.endswith("mixed") else 1e-10)
    else:
        cfg, f = W.tube_batch(n_tubes=40, len_lo=20, len_hi=200, tol=1e-10)
    if "_eq_" in case:
        cfg["regularization"] = "eq"
    if "_sl_" in case:
        cfg["scheme"] = "sl"
    prec = "mixed" if case.endswith("mixed") else "fp64"
    a = pond.Context(cfg, f, precision=prec)
    a.step(11, check=False)
    path = tmp_path / "state.ckpt"
    a.save(path)
    a.step(9, check=False)
    b = pond.Context(cfg, f, precision=prec)
    b.load_state(path)
    b.step(9, check=False)
    assert np.array_equal(a.conserved(), b.conserved())
    assert np.array_equal(a.face_frames(), b.face_frames())
    assert np.array_equal(a.time(), b.time())
    assert np.array_equal(a.failed_instances(), b.failed_instances())


def test_foreign_checkpoint_is_refused(tmp_path):
    from paper_2203_05477_amd import pond

    cfg, f = W.double_mach(32, 16)
    a = pond.Context(cfg, f)
    a.step(2)
    path = tmp_path / "dmr.ckpt"
    a.save(path)
    cfg2, f2 = W.double_mach(32, 16)
    b = pond.Context(cfg2, f2, precision="mixed")  # other precision: other layout
    U0 = b.conserved()
    with pytest.raises(pond.PondError):
        b.load_state(path)
    assert np.array_equal(b.conserved(), U0)
    with pytest.raises(pond.PondError):
        b.load_state(tmp_path / "missing.ckpt")
