"""Host-side behaviour of bench.py (no GPU): the one-GPU guard and the rule
that the committed counter record is used only for the kernel source and rhs
count it was taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_follows_kernel_source(tmp_path, monkeypatch):
    rec = json.load(open(bench.TRAFFIC_FILE))
    val, src = bench.hbm_traffic(rec["nrhs"])
    assert val == rec["bytes_per_launch"] and src.endswith(".json")
    val, why = bench.hbm_traffic(rec["nrhs"] + 1)
    assert val is None and "rhs" in why
    stale = dict(rec, source_sha256="0" * 64)
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    val, why = bench.hbm_traffic(rec["nrhs"])
    assert val is None and "older version" in why
