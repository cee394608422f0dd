"""Host-side checks of the benchmark script: the one-GPU contract and the rocprofv3 summary
arithmetic (counter calibration against the copy kernel), on synthetic counter files."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def _counter_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_profile_summary_calibration(tmp_path, monkeypatch):
    import bench

    h = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))  # the summary goes to tmp_path/profiles
    os.makedirs(tmp_path / "profiles")
    n = 8192
    copy_kib = n * n * 4 / 1024.0
    # the counters report half of the bytes the copy reads, all of those it writes
    rows_f = [{"Kernel_Name": "void fdw::k_copy_out<float>(...)", "Counter_Name": "FETCH_SIZE",
               "Counter_Value": copy_kib / 2}] * 3
    rows_f += [{"Kernel_Name": "void fdw::k_step<float, 8, 2, 0, 5>(fdw::StepArgs)", "Counter_Name": "FETCH_SIZE",
                "Counter_Value": 500000.0}] * 5
    rows_w = [{"Kernel_Name": "void fdw::k_copy_out<float>(...)", "Counter_Name": "WRITE_SIZE",
               "Counter_Value": copy_kib}] * 3
    rows_w += [{"Kernel_Name": "void fdw::k_step<float, 8, 2, 0, 5>(fdw::StepArgs)", "Counter_Name": "WRITE_SIZE",
                "Counter_Value": 540000.0}] * 5
    _counter_csv(str(tmp_path / "f" / "x_counter_collection.csv"), rows_f)
    _counter_csv(str(tmp_path / "w" / "x_counter_collection.csv"), rows_w)
    bench.summarize_profile([str(tmp_path / "f"), str(tmp_path / "w")], "probe", "cmd", "f32")
    js = json.load(open(tmp_path / "profiles" / "probe.json"))
    assert js["fetch_factor"] == pytest.approx(2.0) and js["write_factor"] == pytest.approx(1.0)
    assert js["read_bytes"] == round(500000.0 * 2.0 * 1024)
    assert js["write_bytes"] == round(540000.0 * 1024)
    assert js["algorithmic_bytes"] == 5 * 4 * n * n
    assert js["kernel_source_hash"] == h
    assert "factors fetch 2.0000, write 1.0000" in open(tmp_path / "profiles" / "probe.txt").read()
