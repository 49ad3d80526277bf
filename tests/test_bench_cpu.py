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
    sq = _csv(tmp_path / "sq.csv", [(1, "void k_seg_batch<true, false>(int)", "SQ_INSTS_VALU", 5.0e9),
                                    (1, "void k_seg_batch<true, false>(int)", "SQ_INSTS_LDS", 7.0e8)])
    lds = _csv(tmp_path / "lds.csv", [(1, "void k_seg_batch<true, false>(int)", "SQ_LDS_IDX_ACTIVE", 8.0e8),
                                      (1, "void k_seg_batch<true, false>(int)", "GRBM_GUI_ACTIVE", 1.4e8)])
    bench.pmc_summary(f, w, cf, cw, sq, lds)
    rec = json.load(open(tmp_path / "profiles" / "traffic.json"))["seg_2000x2000"]
    assert rec["sq_lds_idx_active"] == 8.0e8 and rec["grbm_gui_active"] == 1.4e8
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    # the dominant kernel alone
    assert rec["bytes_per_launch"] == pytest.approx((1000.0 * 2.0 + 300.0) * 1024)
    assert rec["sq_insts_valu"] == 5.0e9 and rec["sq_insts_lds"] == 7.0e8
    assert rec["source_hash"] == "h1"
    assert bench._counters("seg_2000x2000")["bytes_per_launch"] == pytest.approx(rec["bytes_per_launch"])
    # measured on other sources: not reported
    monkeypatch.setattr(bench, "_source_hash", lambda: "h2")
    assert bench._counters("seg_2000x2000") is None
    assert bench._counters("no_such_kernel") is None


def test_algorithmic_work_and_issued_mfma_counts():
    import numpy as np
    X = np.zeros((70, 130), order="F")
    X[:, :] = 1.0
    X[5, 3] = 0.0                       # one zero: one 4 x 16 block
    w = bench.algorithmic_work(X)
    assert w["ratio_elements"] == (70 * 130 - 1) * 129
    assert w["residual_terms"] == 70 * 130 * 129
    assert w["flops"] == 2 * w["ratio_elements"] + 3 * w["residual_terms"]
    mf = bench.signsum_mfma_issued(X)
    assert bench.SS_ROWS == 16
    # padded to 80 rows (16-row stages) x 192 columns: 20 x 12 blocks, 3
    # column tiles of 64, 4 waves
    assert mf["mfma_D"] == 20 * 12 * 3 * 4
    # zero blocks: the real zero, every block of padded rows (70..79 -> row
    # blocks 17..19 hold padding: 3 x 12) and of padded columns (130..191:
    # column blocks 8..11 -> 4 x 20), without counting twice
    pad_rows = 3 * 12
    pad_cols = 4 * 20
    both = 3 * 4
    assert mf["mfma_Zr"] == (1 + pad_rows + pad_cols - both) * 3 * 4
