"""Host logic of bench.py that needs no GPU: the traffic summary from two
rocprofv3 --pmc CSVs, and the kernel-source hash that decides whether a
stored traffic figure still describes the kernels."""
import csv
import importlib.util
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod          # dataclasses look their module up there
    spec.loader.exec_module(mod)
    return mod


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_pmc_summary_scales_by_the_copy_pass(bench, tmp_path):
    cfg = bench.CONFIGS["D5"]
    spmv = "cbg::k_spmv_sell<0, true, true>(...)"
    other = "cbg::k_spmv_sell<0, true, false>(...)"      # same pattern, fewer launches
    copy_kib = bench.COPY_CALIB_BYTES / 1024.0
    # the copy pass reads half its bytes on FETCH_SIZE (scale 2) and all on WRITE_SIZE
    _write(tmp_path / "f.csv", "FETCH_SIZE",
           [("at::neg_kernel", copy_kib / 2), (spmv, 1000.0), (spmv, 3000.0), (other, 9e9)])
    _write(tmp_path / "w.csv", "WRITE_SIZE",
           [("at::neg_kernel", copy_kib), (spmv, 10.0), (spmv, 30.0), (other, 9e9)])
    s = bench.pmc_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), cfg)
    assert s["kernel"] == spmv and s["launches"] == [2, 2]
    assert s["fetch_scale"] == 2.0 and s["write_scale"] == 1.0
    assert s["fetch_bytes_per_launch"] == 2000.0 * 1024 * 2.0
    assert s["write_bytes_per_launch"] == 20.0 * 1024
    assert s["traffic_bytes_per_launch"] == 2000.0 * 2048 + 20.0 * 1024
    assert s["kernel_source_sha256"] == bench.kernel_source_hash()


def test_pmc_summary_needs_the_copy_pass(bench, tmp_path):
    cfg = bench.CONFIGS["D2"]
    name = f"cbg::k_multidot<{bench.FMT_ID[cfg.fmt]}, true>(...)"
    _write(tmp_path / "f.csv", "FETCH_SIZE", [(name, 1.0)])
    _write(tmp_path / "w.csv", "WRITE_SIZE", [(name, 1.0)])
    with pytest.raises(SystemExit):
        bench.pmc_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), cfg)


def test_kernel_source_hash_tracks_the_kernel_sources(bench):
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) >= 12
    int(h, 16)


def test_more_than_one_gpu_is_refused(bench, capsys, monkeypatch):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    assert bench.main() != 0
    assert "exactly one GPU" in capsys.readouterr().out
