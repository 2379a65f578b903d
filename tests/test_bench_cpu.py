"""Host logic of bench.py (CPU): the single-GPU contract and the rule that the
committed counter record is reported only for the M2L source it was taken on."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_gate_schedule():
    g = bench.gate_schedule([0, 0, 24, 12, 6], 4, 241, 720)
    assert g[4][0] == 246 and g[4][-1] == 720 and len(g[4]) == 80
    assert len(g[3]) == 40 and len(g[2]) == 20


def test_steady_window_floors():
    """Whatever is requested, the timed steps start after the coarsest level's
    full window and the pulse's arrival, and span whole coarsest intervals."""
    assert bench.steady_window(5, 20, 24, 9, 179) == (216, 24)
    assert bench.steady_window(240, 480, 24, 9, 179) == (240, 480)
    assert bench.steady_window(0, 1, 24, 9, 300) == (312, 24)
    assert bench.steady_window(250, 50, 24, 10, 100) == (264, 72)


def test_physical_cores_is_positive():
    phys, used = bench.physical_cores()
    assert phys >= 1 and 1 <= used <= phys


def test_traffic_record_follows_its_source(tmp_path, monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    got = bench.m2l_traffic("fp64")
    if sha == rec["source_sha256"]:
        assert got == rec["bytes_per_launch"]["fp64"]
    else:
        assert got is None
    assert bench.m2l_traffic("fp32") is None          # no FP32 record
    stale = dict(rec, source_sha256="0" * 64)
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.m2l_traffic("fp64") is None
    fresh = dict(rec, source_sha256=sha)
    p.write_text(json.dumps(fresh))
    assert bench.m2l_traffic("fp64") == rec["bytes_per_launch"]["fp64"]
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.m2l_traffic("fp64") is None
