"""Host-side parts of bench.py that need no GPU: the one-GPU refusal, the
fixed-tiling table (read back by the library's tuning loader), the
roofline's per-launch model and the guard on stored traffic figures."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_fixed_tiling_file_has_one_entry_per_loop_and_class():
    path = bench.fixed_tiling_file("4,0")
    rows = [l.split() for l in open(path)]
    assert len(rows) == 2 * 32
    for r in rows:
        # tag, loop, class, waves, tile, ordered, persistent, split, ms, chunks: the loader's ten fields
        assert r[0] == "best" and len(r) == 10
        assert r[3] == "4" and r[4] == "0"
    assert {(r[1], r[2]) for r in rows} == {(str(m), str(c)) for m in (0, 1) for c in range(32)}


def test_loop_roofline_credits_the_survey_flop_per_interaction():
    bound, per = bench.kernel_model("density_loop", 100, 10, 5, 1000, 2000, 4)
    assert bound == "alu" and per == 54 * 1000 / 4
    bound, per = bench.kernel_model("force_sweep", 100, 10, 5, 1000, 2000, 2)
    assert bound == "alu" and per == 67 * 2000 / 2


def test_stored_traffic_is_dropped_when_its_sources_change(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    import hashlib
    sha = hashlib.sha256(b"kernel v1\n").hexdigest()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "probe", {"bytes": 123.0, "sources": ["k.hip"], "sha256": sha})
    assert bench.measured_traffic("probe") == 123.0
    src.write_text("kernel v2\n")
    assert bench.measured_traffic("probe") is None
    assert bench.measured_traffic("no such kernel") is None
