"""Host-side logic that needs no GPU: the autograd module's surface, the benchmark's refusal of more
than one GPU, and the PMC-record ingestion on synthetic counter files."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_autograd_module_surface():
    from paper_1602_07527_amd import autograd
    for name in ("cholesky", "cholesky_ex", "cholesky_batched", "gp_neg_log_lik"):
        assert callable(getattr(autograd, name))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (k, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Grid_Size": 1024, "Kernel_Name": k, "Counter_Name": counter,
                        "Counter_Value": v})


def test_ingest_pmc_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(tmp_path / "rec.json"))
    tgt = f"void cg::{bench.TARGET_KERNEL}(cg::GemmArgs)"
    narrow = "void cg::gemm_f64_dma_kernel<false, false, 1, 0, false, false>(cg::GemmArgs)"
    cal = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(...)>"
    # The calibration copy of 64 MiB reads as 32768 KiB: every raw value is half the truth.  The
    # 128x128-tile instance of the same contraction is another kernel and is not counted.
    _write_counters(tmp_path / "f.csv", "FETCH_SIZE",
                    [(cal, 32768.0), (tgt, 100.0), (tgt, 300.0), (narrow, 1e9), ("other", 1e9)])
    _write_counters(tmp_path / "w.csv", "WRITE_SIZE", [(cal, 16384.0), (tgt, 50.0)])
    bench.ingest_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 64)
    rec = json.load(open(tmp_path / "rec.json"))
    assert rec["counters"]["FETCH_SIZE"]["scale"] == pytest.approx(2.0)
    assert rec["counters"]["WRITE_SIZE"]["scale"] == pytest.approx(4.0)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(2.0 * 200 * 1024 + 4.0 * 50 * 1024)
    assert bench.traffic_for(bench.source_hashes()) == pytest.approx(rec["hbm_bytes_per_launch"])
    # a changed kernel or a changed launch schedule invalidates the record
    for key in ("kernel_source_sha256", "schedule_source_sha256"):
        assert bench.traffic_for({**bench.source_hashes(), key: "0" * 64}) is None


def test_binding_rejects_unknown_names():
    """Unknown precision / form / diagonal-variant / op names are a ValueError naming the choices,
    raised on the host before any workspace is allocated."""
    from paper_1602_07527_amd import _binding as b
    for table, key, what in ((b._DIAGS, "recursive", "diag"), (b._FORMS, "upper", "form"),
                             (b._PRECS, "bf16", "precision"), (b._OPS, "solve", "op")):
        with pytest.raises(ValueError, match=what):
            b._pick(table, key, what)
    assert b._pick(b._DIAGS, "level2", "diag") == b.DIAG_LEVEL2 == 2
    with pytest.raises(ValueError, match="precision"):
        b.workspace_bytes("rev", 100, precision="f16")
