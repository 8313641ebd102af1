"""Host-side logic of bench.py (no GPU): the one-GPU guard, the calibration of rocprofv3
FETCH_SIZE / WRITE_SIZE counters into bytes per level dispatch, and the rule that a
stored traffic figure is used only for its own workload and unchanged kernel source."""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def _args(**kw):
    a = argparse.Namespace(workload="long", seeds="", bound=0, ruc=False, fkp=False, ucarry=False, udoubling=False)
    for k, v in kw.items():
        setattr(a, k, v)
    return a


def test_workload_key_names_seeds_bound_and_mode():
    assert bench.workload_key(_args()) == "long seeds 0-3 bound 13"
    assert bench.workload_key(_args(workload="scale")) == "scale seeds 0-7 bound 11"
    assert bench.workload_key(_args(workload="hamming", seeds="0-1")) == "hamming seeds 0-1 bound 16"
    assert bench.workload_key(_args(ruc=True, fkp=True)) == "long seeds 0-3 bound 13 ruc fkp"
    assert bench.workload_key(_args(fkp=True)) == "long seeds 0-3 bound 13"   # fkp only with ruc


def _counter_csv(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for did, name, vals in rows:
            for v in vals:      # a counter read per hardware block, summed per dispatch
                w.writerow({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_summarize_counters_calibrates_by_the_copy(tmp_path):
    """The copy of 1 GiB reads and writes 2^20 KiB: the counters are scaled so that it does.
    FETCH_SIZE here reads half of that for the copy (factor 2), WRITE_SIZE all (factor 1);
    only level kernels enter the average, per dispatch."""
    gib_kib = float(1 << 20)
    copy = "__amd_rocclr_copyBuffer"
    lvl = "void ltl::k_level<unsigned long, true, false, 0, false, false>(ltl::LevelArgs<unsigned long>, ...)"
    _counter_csv(tmp_path / "f", "FETCH_SIZE", [
        (1, copy, [gib_kib / 4, gib_kib / 4]),
        (2, lvl, [100.0, 50.0]),
        (3, "k_level_wg<unsigned int, false, false>", [300.0]),
        (4, "k_table_init", [9999.0]),                     # not a level kernel
    ])
    _counter_csv(tmp_path / "w", "WRITE_SIZE", [
        (1, copy, [gib_kib]),
        (2, lvl, [10.0]),
        (3, "k_level_wg<unsigned int, false, false>", [30.0]),
        (4, "k_table_init", [1.0]),
    ])
    out = tmp_path / "t.json"
    bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), "long seeds 0-3 bound 13", str(out))
    rec = json.load(open(out))
    assert rec["calibration"] == {"fetch_factor": 2.0, "write_factor": 1.0}
    assert rec["dispatches"]["level"] == 2
    assert rec["read_bytes_per_launch"] == pytest.approx((150 + 300) * 2 * 1024 / 2)
    assert rec["write_bytes_per_launch"] == pytest.approx((10 + 30) * 1024 / 2)
    assert rec["per_launch_bytes"]["level"] == pytest.approx(((150 + 300) * 2 + 40) * 1024 / 2)
    assert rec["kernel_source_sha256"] == hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()


def test_summarize_counters_needs_the_copy(tmp_path):
    _counter_csv(tmp_path / "f", "FETCH_SIZE", [(2, "k_level<unsigned int>", [1.0])])
    _counter_csv(tmp_path / "w", "WRITE_SIZE", [(2, "k_level<unsigned int>", [1.0])])
    with pytest.raises(SystemExit):
        bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), "k", str(tmp_path / "o.json"))


def test_stored_traffic_only_for_its_workload_and_source(tmp_path, monkeypatch):
    sha = hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()
    good = {"kernel_source_sha256": sha, "workload_key": "long seeds 0-3 bound 13",
            "per_launch_bytes": {"level": 1.5e9}}
    stale = dict(good, kernel_source_sha256="0" * 64, workload_key="scale seeds 0-7 bound 11")
    p1, p2 = tmp_path / "a.json", tmp_path / "b.json"
    p1.write_text(json.dumps(good))
    p2.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TRAFFIC_FILES", [str(p2), str(p1)])
    assert bench.measured_traffic("level", "long seeds 0-3 bound 13") == 1.5e9
    assert bench.measured_traffic("level", "long seeds 0-3 bound 13 ruc") is None
    assert bench.measured_traffic("level", "scale seeds 0-7 bound 11") is None     # source changed since
    assert bench.measured_traffic("verify", "long seeds 0-3 bound 13") is None
