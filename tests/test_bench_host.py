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
    """A counter record is used only while the kernel source, the rhs count
    and the link format / coarse operator match the run (a record written
    here for the current source; the committed one is used the same way)."""
    import hashlib
    sha = hashlib.sha256(open(bench.DOM_SOURCE, "rb").read()).hexdigest()
    mode = bench.coarse_mode("bf16", 1)
    rec = {"nrhs": 64, "mode": mode, "source_sha256": sha, "bytes_per_launch": 1.5e9}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    val, src = bench.hbm_traffic(64, mode)
    assert val == 1.5e9 and src.endswith(".json")
    val, why = bench.hbm_traffic(65, mode)
    assert val is None and "rhs" in why
    val, why = bench.hbm_traffic(64, bench.coarse_mode("fp16", 1))
    assert val is None and mode in why
    f.write_text(json.dumps(dict(rec, source_sha256="0" * 64)))
    val, why = bench.hbm_traffic(64, mode)
    assert val is None and "older version" in why
