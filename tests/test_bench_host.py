"""Host logic of the measurement (no GPU): the roofline's algorithmic units,
the reading of committed traffic summaries, and the scaling of rocprofv3
counters by a plain copy."""
import csv

import pytest

import bench
from paper_2303_12873_amd import profsum

C5_PARTICLES = 1_010_827_264        # 2 species x 4 per cell where the plasma is (vacuum, ramp)
C5_CELLS = 134_217_728


def test_roofline_units_of_the_split_particle_kernel():
    # per particle 60 B (int32 cell, 3 offsets, 3 momenta, weight read; cell,
    # offsets, momenta written), per cell 48 B (E, B FP32 read, J FP64
    # written), 2,150 flops per particle at order 3
    assert C5_CELLS == 256 * 256 * 2048 and C5_PARTICLES < 2 * 4 * C5_CELLS
    r = bench.roofline(C5_PARTICLES, C5_CELLS, 3, True, "fp32", 100.0, bound="alu")
    assert r["algorithmic_bytes_per_launch"] == C5_PARTICLES * 60 + C5_CELLS * 48 == 67_092_086_784
    assert r["algorithmic_flops_per_launch"] == C5_PARTICLES * 2150
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["achieved"] == pytest.approx(C5_PARTICLES * 2150 / 0.1 / 1e12, abs=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6, abs=1e-4)
    assert r["hbm_frac"] == pytest.approx(67_092_086_784 / 0.1 / 8e12, abs=1e-4)


def test_roofline_units_of_the_fp64_hbm_workload():
    # C2-sized box, 128 x 128 x 1024 cells, counted as 2 particles in every
    # cell; FP64 104 B per particle, 72 B per cell
    n, cells = 2 * 128 * 128 * 1024, 128 * 128 * 1024
    r = bench.roofline(n, cells, 2, True, "fp64", 5.0, bound="hbm")
    assert r["algorithmic_bytes_per_launch"] == n * 104 + cells * 72
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx((n * 104 + cells * 72) / 5e-3 / 1e9, abs=0.1)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    # a bound is chosen by the larger fraction when none is named
    assert bench.roofline(n, cells, 2, True, "fp64", 5.0)["bound"] == "hbm"


def test_fdtd_roofline_bytes_per_cell():
    r = bench.fdtd_roofline(1000, "fp32", 1.0)
    assert r["algorithmic_bytes"] == 72 * 1000 and r["bytes_three_passes"] == 132 * 1000
    r = bench.fdtd_roofline(1000, "fp64", 1.0)
    assert r["algorithmic_bytes"] == 120 * 1000 and r["bytes_three_passes"] == 240 * 1000


def _summary(path, workload, config, sha, value):
    path.write_text(f"# summary\n\n- workload: {workload}\n- config: {config}\n"
                    f"- kernel_source_sha256: {sha}\n- traffic_bytes_per_launch: {value}\n")


def test_measured_traffic_only_for_its_own_run(tmp_path):
    sha = bench.kernel_source_sha()
    cfg = "tile=(16, 8, 4) block=1024 lane_stride=1 cell_order=4 pad=0 margin=0"
    p = tmp_path / "t.md"
    _summary(p, "w", cfg, sha, 123)
    assert bench.measured_traffic("w", cfg, str(p)) == 123
    assert bench.measured_traffic("other", cfg, str(p)) is None
    assert bench.measured_traffic("w", cfg.replace("block=1024", "block=512"), str(p)) is None
    _summary(p, "w", cfg, "0" * 64, 123)          # taken with other kernel sources
    assert bench.measured_traffic("w", cfg, str(p)) is None
    _summary(p, "w", cfg, sha, "n/a")
    assert bench.measured_traffic("w", cfg, str(p)) is None
    assert bench.measured_traffic("w", cfg, str(tmp_path / "missing.md")) is None


def test_launch_config_string():
    from paper_2303_12873_amd.autotune import Candidate
    c = Candidate((16, 8, 4), 1024, 8192, 2, 1, 4, 16, 0, 0)
    assert bench.launch_config(c) == "tile=(16, 8, 4) block=1024 lane_stride=1 cell_order=4 pad=0 margin=0"


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_scaled_by_a_plain_copy(tmp_path):
    # the copy of B bytes reads FETCH_SIZE = B / 2 and WRITE_SIZE = B (KiB)
    B = 4 * 2**30
    _counter_csv(tmp_path / "cf.csv", [("k_copy16(...)", "FETCH_SIZE", B / 2 / 1024)] * 2)
    _counter_csv(tmp_path / "cw.csv", [("k_copy16(...)", "WRITE_SIZE", B / 1024)] * 2)
    _counter_csv(tmp_path / "f.csv", [("k_tiled<X>(...)", "FETCH_SIZE", 1000.0),
                                      ("k_tiled<X>(...)", "FETCH_SIZE", 3000.0),
                                      ("k_other(...)", "FETCH_SIZE", 9e9)])
    _counter_csv(tmp_path / "w.csv", [("k_tiled<X>(...)", "WRITE_SIZE", 500.0),
                                      ("k_tiled<X>(...)", "WRITE_SIZE", 500.0)])
    r = profsum.traffic(tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "cf.csv",
                        tmp_path / "cw.csv", B, "k_tiled<X>")
    assert r["fetch_scale"] == pytest.approx(2.0) and r["write_scale"] == pytest.approx(1.0)
    assert r["fetch_bytes"] == pytest.approx(2000.0 * 1024 * 2)
    assert r["write_bytes"] == pytest.approx(500.0 * 1024)
    assert r["traffic_bytes_per_launch"] == 2000 * 1024 * 2 + 500 * 1024
    assert r["dispatches"] == (2, 2)
    with pytest.raises(SystemExit):
        profsum.traffic(tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "cf.csv",
                        tmp_path / "cw.csv", B, "k_absent")
