"""Host-side pieces of bench.py: the HBM byte count from rocprofv3 counter
files (FETCH_SIZE / WRITE_SIZE per dispatch, scaled by a copy of known size)
and the refusal of more than one GPU.  No GPU is used."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for did, name, value in rows:
            # rocprofv3 may split a counter over several rows of a dispatch
            w.writerow({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value / 2})
            w.writerow({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value / 2})


def test_traffic_from_counters(tmp_path):
    copy = "void at::native::vectorized_elementwise_kernel<4, MulFunctor>(int)"
    giant = "eis::k_walk_giant(eis::InfraParams)"
    window = "eis::k_walk_window(eis::InfraParams)"
    # the copy of 1024 MiB reads half its bytes by FETCH_SIZE (scale 2), writes them all
    _write_counters(tmp_path / "f", "FETCH_SIZE",
                    [(1, copy, 512 * 1024), (7, giant, 1000.0), (9, giant, 3000.0),
                     (5, window, 50.0)])
    _write_counters(tmp_path / "w", "WRITE_SIZE",
                    [(1, copy, 1024 * 1024), (7, giant, 10.0), (9, giant, 30.0),
                     (5, window, 800.0)])
    per, probe = bench.traffic_from_counters(str(tmp_path / "f"), str(tmp_path / "w"), 1024)
    assert probe["fetch_scale"] == pytest.approx(2.0) and probe["write_scale"] == pytest.approx(1.0)
    # the last dispatch of each kernel, in KiB, scaled, in bytes
    assert per["k_walk_giant"] == (3000.0, 30.0, int((3000.0 * 2 + 30.0) * 1024))
    assert per["k_walk_window"] == (50.0, 800.0, int((50.0 * 2 + 800.0) * 1024))
    assert "k_build_tables" not in per


def test_traffic_from_counters_needs_files(tmp_path):
    with pytest.raises(RuntimeError):
        bench.traffic_from_counters(str(tmp_path / "none"), str(tmp_path / "none"), 1024)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
