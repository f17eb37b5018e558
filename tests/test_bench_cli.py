"""bench.py on a machine without a GPU: more than one GPU is refused with a message, the HBM
traffic figure is read from the committed counter summary only while the kernel sources still
hash to the value recorded there, and a timed window runs without per-kernel events while its
twin takes the kernel times."""
import hashlib
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr


def test_traffic_figure_follows_the_source_hash():
    sys.path.insert(0, ROOT)
    import bench

    txt = open(bench.TRAFFIC_PROFILE).read()
    recs = [json.loads(m) for m in re.findall(r"traffic-json: (\{.*\})", txt)]
    assert recs
    src = b"".join(open(os.path.join(ROOT, "paper_2203_05477_amd", "csrc", f), "rb").read()
                   for f in bench.KERNEL_SOURCES)
    for rec in recs:
        same = hashlib.sha256(src).hexdigest() == rec["sources_sha256"]
        got = bench.measured_traffic(rec["tiles"])
        if same:
            assert got is not None and got["bytes_per_launch"] == rec["bytes_per_launch"] > 0
        else:
            assert got is None
    assert bench.measured_traffic([7, 3]) is None  # no record for a tile never measured


def test_tube_traffic_follows_the_source_hash():
    sys.path.insert(0, ROOT)
    import bench

    txt = open(bench.TUBE_TRAFFIC_PROFILE).read()
    recs = [json.loads(m) for m in re.findall(r"traffic-json: (\{.*\})", txt)]
    assert len(recs) == 2
    src = b"".join(open(os.path.join(ROOT, "paper_2203_05477_amd", "csrc", f), "rb").read()
                   for f in bench.KERNEL_SOURCES)
    for rec in recs:
        got = bench.tube_traffic(rec["kernel"])
        if hashlib.sha256(src).hexdigest() == rec["sources_sha256"]:
            assert got == rec["bytes_per_cell_update"] > 0
        else:
            assert got is None
    assert bench.tube_traffic("no such kernel") is None


class _FakeContext:
    """Stands in for pond.Context in timed_steps: steps advance a counter, the state is that
    counter (or a planted difference), and kernel times exist only while timing is on."""

    def __init__(self, offset=0.0):
        self.n, self.offset, self.timing, self.calls = 0, offset, None, []

    def enable_timing(self, on=True):
        self.timing = bool(on)
        self.calls.append(("timing", bool(on)))

    def step(self, k, check=True):
        self.calls.append(("step", k))
        self.n += k
        return {"converged_cell_updates": 10 * k, "cell_updates": 10 * k}

    def conserved(self):
        import numpy as np

        return np.full((4, 3), float(self.n) + self.offset)

    def kernel_times(self):
        assert self.timing, "kernel times asked of a context without events"
        return {"dt": 0.001, "face": 0.1, "tail": 0.05, "cell": 0.01, "seed": 0.0}


def test_timed_window_runs_without_events_and_its_twin_with_them(monkeypatch):
    """The rate comes from a window with the per-kernel events off; the kernel times from a
    twin with them on, which must end in the same state (a twin that does not is reported)."""
    sys.path.insert(0, ROOT)
    import bench
    import torch

    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    ctx, twin = _FakeContext(), _FakeContext()
    st, el, U, kt, rec = bench.timed_steps(ctx, 7, twin)
    assert ctx.calls[0] == ("timing", False) and ("step", 7) in ctx.calls
    assert twin.calls[0] == ("timing", True) and ("step", 7) in twin.calls
    assert st["cell_updates"] == 70 and el >= 0.0 and U[0, 0] == 7.0
    assert kt["face"] == 0.1 and rec["same_state"] is True and rec["ms_per_step_with_events"] >= 0.0
    _, _, _, _, rec = bench.timed_steps(_FakeContext(), 3, _FakeContext(offset=1e-12))
    assert rec["same_state"] is False
    _, _, _, kt, rec = bench.timed_steps(_FakeContext(), 3)
    assert kt is None and rec is None
