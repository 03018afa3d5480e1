"""bench.py on the CPU: the one-GPU contract and the traffic records.

* `--gpus` above 1 exits with status 2 and a message (the benchmark
  measures one GPU; the multi-GPU decomposition is a design note).
* The committed HBM traffic records (profiles/traffic.json) are looked up
  only when they were taken on the current kernel source: a record whose
  source hash differs reads as None, so a stale counter figure never reaches
  the benchmark line.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_records_are_current():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for s in (1, 2, 3, 4):
        ent = rec["1d_2048x378"][f"stage{s}"]
        assert ent["source_hash"] == bench.kernel_source_hash()
        assert bench.measured_traffic(f"stage{s}", "1d_2048x378") == ent["bytes_per_launch"]
        # HBM bytes within a few percent above the algorithmic bytes
        assert 1.0 <= ent["bytes_per_launch"] / ent["alg_bytes"] < 1.2
    for wl, hfun in (("3d_64x92", bench.source_hash_3d), ("batch_64_uneven", bench.kernel_source_hash)):
        for k, ent in rec[wl].items():
            assert ent["source_hash"] == hfun(), (wl, k)
            # a record is used only in the launch shape it was taken at
            assert bench.measured_traffic(k, wl, hfun(), launch=ent["launch"]) == ent["bytes_per_launch"]
            other = dict(ent["launch"], steps_per_graph=ent["launch"]["steps_per_graph"] + 1)
            assert bench.measured_traffic(k, wl, hfun(), launch=other) is None
            assert 0.95 <= ent["bytes_per_launch"] / ent["alg_bytes"] < 1.2, (wl, k)
    h = bench.particles_source_hash()
    for k, ent in rec["1d_2048x378_random"].items():
        assert ent["source_hash"] == h, k
        assert bench.measured_traffic(k, "1d_2048x378_random", h) == ent["bytes_per_launch"]


def test_stale_traffic_record_reads_as_none(tmp_path, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    rec["1d_2048x378"]["stage4"]["source_hash"] = "0" * 16
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "1" * 16)
    assert bench.measured_traffic("stage4", "1d_2048x378") is None
    assert bench.measured_traffic("stage9", "1d_2048x378") is None
    assert bench.measured_traffic("stage4", "no_such_box") is None


@pytest.mark.parametrize("s,expect", [(1, 272), (2, 400), (3, 400), (4, 672)])
def test_stage_bytes(s, expect):
    # state 18 reals, slopes 16 reals (traceless), per particle and stage
    assert bench.STAGE_BYTES[s] == expect
    assert sum(bench.STAGE_BYTES[k] for k in (1, 2, 3, 4)) == 1744
