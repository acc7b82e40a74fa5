"""Host arithmetic behind the measured figures (no GPU): the calibration of
the FETCH_SIZE / WRITE_SIZE counters by a copy of known size, the traffic
record that bench.py reports only for unchanged kernel sources, and the MFMA
and HBM tables built from counter dumps.  The counter dumps are small
synthetic files in rocprofv3's csv layout."""
import csv
import json

import pytest

import bench
import bench_profile

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
          "End_Timestamp"]


def _dump(path, rows):
    """rows: (dispatch, kernel, counter, value, start ns, end ns); one file
    as rocprofv3 writes it (counter values may come split over instances)."""
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(FIELDS)
        for r in rows:
            w.writerow(r)
    return str(path)


def test_traffic_calibration(tmp_path):
    # a 1 MiB copy counted as 512 KiB read (in two instances) and 1024 KiB
    # written: 2 and 1 bytes per counted byte
    fetch = _dump(tmp_path / "f.csv", [
        (1, "neg_kernel<double>", "FETCH_SIZE", 256, 0, 10),
        (1, "neg_kernel<double>", "FETCH_SIZE", 256, 0, 10),
        (2, "k_large_persist<32,false>", "FETCH_SIZE", 1000, 10, 20),
        (3, "k_large_persist<32,false>", "FETCH_SIZE", 3000, 20, 30),
        (4, "k_other", "FETCH_SIZE", 99999, 30, 40)])
    write = _dump(tmp_path / "w.csv", [
        (1, "neg_kernel<double>", "WRITE_SIZE", 1024, 0, 10),
        (2, "k_large_persist<32,false>", "WRITE_SIZE", 500, 10, 20),
        (3, "k_large_persist<32,false>", "WRITE_SIZE", 700, 20, 30)])
    t = bench_profile.traffic(fetch, write, "k_large_persist", "w1", 1)
    f, wr = t["counters"]["FETCH_SIZE"], t["counters"]["WRITE_SIZE"]
    assert f["launches"] == 2 and f["calibration_kib"] == 512
    assert f["bytes_per_kib"] == pytest.approx(2048.0)
    assert f["bytes_per_launch"] == pytest.approx(2000 * 2048.0)
    assert wr["bytes_per_kib"] == pytest.approx(1024.0)
    assert wr["bytes_per_launch"] == pytest.approx(600 * 1024.0)
    assert t["hbm_bytes_per_launch"] == pytest.approx(2000 * 2048.0 + 600 * 1024.0)
    assert t["source_sha256"] == bench.f_kernel_hash() and t["workload"] == "w1"


def test_traffic_record_needs_the_same_sources_and_workload(tmp_path):
    p = tmp_path / "t.json"
    assert bench.measured_traffic(str(p), "w1") is None  # no record
    p.write_text(json.dumps({"source_sha256": bench.f_kernel_hash(), "workload": "w1",
                             "hbm_bytes_per_launch": 5.0}))
    assert bench.measured_traffic(str(p), "w1")["hbm_bytes_per_launch"] == 5.0
    assert bench.measured_traffic(str(p), "w2") is None
    p.write_text(json.dumps({"source_sha256": "0" * 64, "workload": "w1"}))
    assert bench.measured_traffic(str(p), "w1") is None
    p.write_text("not json")
    assert bench.measured_traffic(str(p), "w1") is None


def test_mfma_table(tmp_path):
    # 1e9 BF16 MOPS = 512e9 flops in 1 ms; busy 1000 cycles against 8000
    # active cycles summed over 8 XCDs on 1024 SIMDs
    d = _dump(tmp_path / "m.csv", [
        (7, "k_mlp_bf16<256>", "SQ_INSTS_VALU_MFMA_MOPS_BF16", 1e9, 0, 1_000_000),
        (7, "k_mlp_bf16<256>", "SQ_VALU_MFMA_BUSY_CYCLES", 1000, 0, 1_000_000),
        (7, "k_mlp_bf16<256>", "GRBM_GUI_ACTIVE", 8000, 0, 1_000_000)])
    row = [l for l in bench_profile.mfma_table(d, ["k_mlp_bf16"]).splitlines()
           if l.startswith("| `k_mlp_bf16`")][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1] == "1"
    assert float(cells[2]) == pytest.approx(0.512)
    assert float(cells[3]) == pytest.approx(1000 / (1000 * 1024), abs=1e-4)
    assert float(cells[4]) == pytest.approx(512.0)


def test_hbm_table(tmp_path):
    # calibration 1 MiB counted as 1024 units (1024 bytes per unit); the
    # kernel reads 2000 and writes 1000 units in 2 us
    f = _dump(tmp_path / "f.csv", [(1, "neg_kernel", "FETCH_SIZE", 1024, 0, 5),
                                   (2, "k_batch_fine", "FETCH_SIZE", 2000, 100, 2100)])
    w = _dump(tmp_path / "w.csv", [(1, "neg_kernel", "WRITE_SIZE", 1024, 0, 5),
                                   (2, "k_batch_fine", "WRITE_SIZE", 1000, 100, 2100)])
    row = [l for l in bench_profile.hbm_table(f, w, ["k_batch_fine"], 1).splitlines()
           if l.startswith("| `k_batch_fine`")][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1] == "1"
    assert float(cells[2]) == pytest.approx(2000 * 1024 / 1e9, abs=1e-3)
    assert float(cells[3]) == pytest.approx(1000 * 1024 / 1e9, abs=1e-3)
    assert float(cells[5]) == pytest.approx(3000 * 1024 / 2000, rel=1e-3)
