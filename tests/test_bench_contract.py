"""bench.py's command-line contract that can be checked without a GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_entries_are_ignored_once_the_kernel_source_changes(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    os.makedirs(tmp_path / "paper_2103_11991_amd" / "csrc")
    for f in ("spg_accum.hip", "spg_internal.h"):
        (tmp_path / "paper_2103_11991_amd" / "csrc" / f).write_text("v1 " + f)
    sha = bench.kernel_source_sha()
    (tmp_path / "profiles" / "traffic.json").write_text(
        json.dumps({"num_class_14": {"source_sha": sha, "hbm_bytes_per_launch": 123.0}}))
    assert bench.stored_traffic("num_class_14") == 123.0
    (tmp_path / "paper_2103_11991_amd" / "csrc" / "spg_accum.hip").write_text("v2")
    assert bench.stored_traffic("num_class_14") is None
