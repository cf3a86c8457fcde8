"""CPU: the host-side bookkeeping of bench.py (no GPU): HBM counter summaries scaled by the
calibration copy, their kernel-source stamp, and the uneven-batch parameter rule."""
import csv
import json
import os

import pytest

import bench

FIELDS = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def write_rows(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for name, grid, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter, "Counter_Value": value})


@pytest.fixture
def traffic_file(tmp_path, monkeypatch):
    path = tmp_path / "profiles" / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    return path


def test_counters_scaled_by_the_calibration_copy(tmp_path, traffic_file):
    sweep = "void pgm::k_sweep<6, 8, true, 0>(pgm::SweepArgs)"
    other = "void pgm::k_sweep<6, 16, false, 0>(pgm::SweepArgs)"
    copy = "__amd_rocclr_copyBuffer"
    # a 256 MiB copy: FETCH_SIZE counts half of it (KiB), WRITE_SIZE all of it
    write_rows(tmp_path / "f.csv", "FETCH_SIZE", [(copy, 1, 131072.0), (sweep, 1, 3000.0), (sweep, 1, 5000.0),
                                                  (other, 1, 1e9)])
    write_rows(tmp_path / "w.csv", "WRITE_SIZE", [(copy, 1, 262144.0), (sweep, 1, 40.0), (sweep, 1, 60.0)])
    bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 256)
    t = json.loads(traffic_file.read_text())
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert t["fetch_bytes_per_launch"] == 2 * 1024 * 4000      # other variants are not counted
    assert t["write_bytes_per_launch"] == 1024 * 50
    assert t["launches"] == 2
    assert bench.measured_traffic() == 2 * 1024 * 4000 + 1024 * 50


def test_traffic_is_dropped_when_the_kernels_change(traffic_file):
    os.makedirs(traffic_file.parent, exist_ok=True)
    traffic_file.write_text(json.dumps({"fetch_bytes_per_launch": 1, "write_bytes_per_launch": 2,
                                        "kernel_source_sha256": "0" * 64}))
    assert bench.measured_traffic() is None
    traffic_file.write_text(json.dumps({"fetch_bytes_per_launch": 1, "write_bytes_per_launch": 2,
                                        "kernel_source_sha256": bench._source_hash()}))
    assert bench.measured_traffic() == 3


def test_missing_calibration_copy_is_an_error(tmp_path, traffic_file):
    sweep = "void pgm::k_sweep<6, 8, true, 0>(pgm::SweepArgs)"
    write_rows(tmp_path / "f.csv", "FETCH_SIZE", [(sweep, 1, 1.0)])
    write_rows(tmp_path / "w.csv", "WRITE_SIZE", [(sweep, 1, 1.0)])
    with pytest.raises(SystemExit):
        bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 256)


def test_uneven_batch_parameters_bound_the_displacement_by_a_fifth_of_the_width():
    import oracle
    import paper_1704_03217_amd as pgm
    for preset in (None, pgm.PRESET_CONFIG5):
        for w, h, d in ((320, 240, 64), (640, 480, 128), (1024, 436, 205), (1242, 375, 249)):
            p = bench.sized_params(pgm, w, preset)
            assert p.max_disp == -5 and p.levels == 5 and p.seed_stride == 3
            explicit = dict(pgm.params_dict(p), max_disp=d)
            assert oracle.top_radius(pgm.params_dict(p), w, h) == oracle.top_radius(explicit, w, h)


def test_all_core_oracle_baseline_reports_its_sample():
    import paper_1704_03217_amd as pgm
    r = bench.cpu_all_cores(pgm.params_dict(pgm.pgm_default_params(pgm.PRESET_CONFIG1)), 0.5, config=1)
    assert r["cores"] == r["processes"] >= 1 and r["runs"] >= r["processes"] and r["value"] > 0
    assert "independent" in r["sample"]
