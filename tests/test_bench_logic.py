"""Host logic of bench.py that needs no GPU: algorithmic bytes, the tile shape read from
a kernel name, and the HBM-traffic summary of two rocprofv3 counter runs (scaled by the
copy kernel's reading, keyed by kernel sources, workload and tile shape)."""
import csv
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes():
    # five passes of nvar FP64 values per cell-update: read U, write U1; read U1 and U, write U
    assert bench.bytes_per_cell(5) == 200 and bench.bytes_per_cell(8) == 320 and bench.bytes_per_cell(9) == 360
    assert bench.bytes_stage(5) == (80, 120)
    assert sum(bench.bytes_stage(8)) == bench.bytes_per_cell(8)


def test_stage_tile_from_kernel_names():
    assert bench.stage_tile("void amr::stage_kernel<float, 5, 32, 16, 512, 2, false, true>(amr::StageArgs)") == "32x16"
    assert bench.stage_tile("void amr::stage_kernel<double, 8, 0, 0, 256, 1, true, true>(amr::StageArgs)") == "0x0"
    assert bench.stage_tile("amr::copy_ghosts(amr::CopyOp const*)") is None


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_summary_scales_by_the_copy_and_keys_the_entry(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    copy = "__amd_rocclr_copyBuffer"
    s1 = "void amr::stage_kernel<float, 5, 32, 16, 512, 1, false, true>(amr::StageArgs)"
    s2 = "void amr::stage_kernel<float, 5, 32, 16, 512, 2, false, true>(amr::StageArgs)"
    other = "void amr::stage_kernel<float, 5, 8, 8, 256, 1, false, true>(amr::StageArgs)"  # a tuning candidate
    gib_kib = (1 << 30) / 1024.0
    # the counters read the 1 GiB copy as half its reads and all of its writes
    _counter_csv(tmp_path / "F.csv", "FETCH_SIZE",
                 [(copy, gib_kib / 2), (s1, 100.0), (s1, 300.0), (s1, 200.0), (s2, 400.0), (s2, 400.0),
                  (other, 9999.0)])
    _counter_csv(tmp_path / "W.csv", "WRITE_SIZE",
                 [(copy, gib_kib), (s1, 50.0), (s1, 50.0), (s1, 50.0), (s2, 60.0), (s2, 60.0), (other, 1.0)])
    cells = 1000
    e = bench.summarize_pmc(str(tmp_path / "F.csv"), str(tmp_path / "W.csv"), "box", "batched_mixed", cells)
    assert e["copy_scale_fetch"] == pytest.approx(2.0) and e["copy_scale_write"] == pytest.approx(1.0)
    assert e["tile"] == "32x16" and set(e["kernels"]) == {s1, s2}  # the shape with the most dispatches
    # medians x 1024 x scale: stage 1 200 KiB read, 50 written; stage 2 400 and 60
    assert e["kernels"][s1]["fetch_bytes"] == pytest.approx(200 * 1024 * 2.0)
    assert e["kernels"][s2]["write_bytes"] == pytest.approx(60 * 1024)
    per_launch = ((200 * 2 + 50) + (400 * 2 + 60)) * 1024 / 2
    assert e["hbm_bytes_per_launch"] == pytest.approx(per_launch)
    assert e["algorithmic_bytes_per_launch"] == pytest.approx(200 * cells / 2)
    assert bench.traffic_for("box", "batched_mixed", cells, "32x16") == pytest.approx(per_launch)
    # any other workload size, tile shape or kernel sources: no measurement
    assert bench.traffic_for("box", "batched_mixed", cells + 1, "32x16") is None
    assert bench.traffic_for("box", "batched_mixed", cells, "8x8") is None
    assert bench.traffic_for("box", "batched_fp64", cells, "32x16") is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 16)
    assert bench.traffic_for("box", "batched_mixed", cells, "32x16") is None


def test_kernel_source_hash_is_stable_and_covers_the_tile_host_code():
    assert bench.kernel_source_sha() == bench.kernel_source_sha()
    assert "amr_stage.h" in bench.STAGE_SOURCES and "amr_api.hip" in bench.STAGE_SOURCES
