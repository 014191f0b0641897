"""Host logic of bench.py, on the CPU: the one-GPU guard, the parsing of rocprofv3 counter
files, and the gating of the committed traffic record (a record counts only for the solver
configuration and the kernel sources it was taken with)."""

import copy
import csv
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_counter_mean_per_dispatch(tmp_path):
    path = tmp_path / "c.csv"
    rows = [  # a dispatch's counter can come in several rows (one per block of the chip): they add up
        (1, "void k_x<1>(int)", "FETCH_SIZE", 1.0), (1, "void k_x<1>(int)", "FETCH_SIZE", 2.0),
        (2, "void k_x<1>(int)", "FETCH_SIZE", 3.0), (2, "void k_x<1>(int)", "FETCH_SIZE", 4.0),
        (2, "void k_x<1>(int)", "WRITE_SIZE", 100.0), (3, "void k_y(int)", "FETCH_SIZE", 50.0),
    ]
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writerows(rows)
    mean, n = bench._counter_kib_per_dispatch(str(path), "FETCH_SIZE", "k_x")
    assert n == 2 and mean == 5.0
    mean, n = bench._counter_kib_per_dispatch(str(path), "WRITE_SIZE", "k_x")
    assert n == 1 and mean == 100.0


def test_traffic_record_gating(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    args = bench.parse()
    with open(os.path.join(ROOT, "profiles", "traffic_k_trsv_sweep_c2.json")) as f:
        rec = json.load(f)
    current = bench._sources_sha256(rec["sources"]) == rec["sources_sha256"]
    same_cfg = all(getattr(args, k) == v for k, v in rec["config"].items())
    got = bench.measured_traffic("k_trsv_sweep", "c2", args)
    assert got == (rec["traffic_bytes_per_launch"] if current and same_cfg else None)
    # the record of the default configuration counts for no other one
    for key, value in (("cg_steps", args.cg_steps + 1), ("p", args.p + 1), ("precision", "fp32"), ("ytau", 0.5)):
        other = copy.copy(args)
        setattr(other, key, value)
        assert bench.measured_traffic("k_trsv_sweep", "c2", other) is None, key
    assert bench.measured_traffic("k_no_such_kernel", "c2", args) is None
