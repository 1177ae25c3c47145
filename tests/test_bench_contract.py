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


def _pmc_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "pmc_counter_collection.csv"), "w") as fh:
        fh.write('"Dispatch_Id","Grid_Size","Kernel_Name","Counter_Name","Counter_Value"\n')
        for d, g, k, c, v in rows:
            fh.write(f'{d},{g},"{k}","{c}",{v}\n')


def test_counter_summary_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    """FETCH_SIZE and WRITE_SIZE of the largest-grid numeric dispatches, each
    scaled so that the 1 GiB copy reads as 1 GiB."""
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "paper_2103_11991_amd" / "csrc")
    for f in ("spg_accum.hip", "spg_internal.h"):
        (tmp_path / "paper_2103_11991_amd" / "csrc" / f).write_text("src " + f)
    k, small = "void k_num<64, 2, double>(NumArgs)", "void k_num<32, 2, double>(NumArgs)"
    _pmc_csv(tmp_path / "f", [(1, 1000, k, "FETCH_SIZE", 100.0), (2, 1000, k, "FETCH_SIZE", 300.0),
                              (3, 10, small, "FETCH_SIZE", 7.0)])
    _pmc_csv(tmp_path / "w", [(1, 1000, k, "WRITE_SIZE", 50.0), (2, 1000, k, "WRITE_SIZE", 50.0)])
    _pmc_csv(tmp_path / "cf", [(1, 512, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0)])
    _pmc_csv(tmp_path / "cw", [(1, 512, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0)])
    ent = bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                                   str(tmp_path / "cw"), cls=23, command="x")
    assert ent["fetch"]["scale"] == 2.0 and ent["write"]["scale"] == 1.0
    assert ent["hbm_bytes_per_launch"] == 200.0 * 1024 * 2 + 50.0 * 1024
    assert bench.stored_traffic("num_class_23") == ent["hbm_bytes_per_launch"]
