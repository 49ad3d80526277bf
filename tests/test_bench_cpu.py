"""Host logic of bench.py (no GPU): the one-GPU guard, the counter-file
parsing, the HBM-traffic summary scaled by the copy calibration, and the
rule that stored traffic is reported only for the kernel sources it was
measured on."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], r)))
    return str(path)


def test_counter_parsing_per_dispatch(tmp_path):
    # two dispatches of a templated kernel, one counter row per XCD each
    rows = [(1, "void k_seg_batch<true, false>(ProbDesc const*)", "FETCH_SIZE", 10.0),
            (1, "void k_seg_batch<true, false>(ProbDesc const*)", "FETCH_SIZE", 30.0),
            (2, "void k_seg_batch<true, false>(ProbDesc const*)", "FETCH_SIZE", 20.0),
            (2, "void k_seg_batch<true, false>(ProbDesc const*)", "FETCH_SIZE", 20.0),
            (2, "void k_seg_batch<true, false>(ProbDesc const*)", "WRITE_SIZE", 99.0),
            (3, "k_signsum_batch(ProbDesc const*, int)", "FETCH_SIZE", 7.0)]
    got = bench._pmc_per_dispatch(_csv(tmp_path / "c.csv", rows), "FETCH_SIZE")
    assert got == {"k_seg_batch": 40.0, "k_signsum_batch": 7.0}


def test_traffic_summary_and_source_rule(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_source_hash", lambda: "h1")
    copy = "__amd_rocclr_copyBuffer"
    kib = (512 << 20) / 1024
    # the copy of 512 MiB reads as half its bytes on FETCH_SIZE, in full on WRITE_SIZE
    cf = _csv(tmp_path / "cf.csv", [(1, copy, "FETCH_SIZE", kib / 2)])
    cw = _csv(tmp_path / "cw.csv", [(1, copy, "WRITE_SIZE", kib)])
    f = _csv(tmp_path / "f.csv", [(1, "void k_seg_batch<true, false>(int)", "FETCH_SIZE", 1000.0),
                                  (1, "k_signsum_batch(int)", "FETCH_SIZE", 100.0)])
    w = _csv(tmp_path / "w.csv", [(1, "void k_seg_batch<true, false>(int)", "WRITE_SIZE", 300.0),
                                  (1, "k_signsum_batch(int)", "WRITE_SIZE", 60.0)])
    bench.pmc_summary(f, w, cf, cw)
    rec = json.load(open(tmp_path / "profiles" / "traffic.json"))["seg_2000x2000"]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["bytes_per_launch"] == pytest.approx((1100.0 * 2.0 + 360.0) * 1024)
    assert rec["source_hash"] == "h1"
    assert bench._traffic("seg_2000x2000") == pytest.approx(rec["bytes_per_launch"])
    # measured on other sources: not reported
    monkeypatch.setattr(bench, "_source_hash", lambda: "h2")
    assert bench._traffic("seg_2000x2000") is None
    assert bench._traffic("no_such_kernel") is None
