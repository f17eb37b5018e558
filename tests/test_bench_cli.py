"""bench.py's command line on a machine without a GPU: more than one GPU is refused with a
message, and the HBM traffic figure is read from the committed counter summary only while
the kernel sources still hash to the value recorded there."""
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
