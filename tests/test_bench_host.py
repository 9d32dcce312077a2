"""Host logic of bench.py (no GPU): the flop model, the roofline records, the
traffic table's keying, and the one-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_flop_model_values_quoted_for_the_workloads():
    # C2 (N=3, K=3, isotropic, 2D) and C3 (N=2, K=2, anisotropic, 3D)
    assert bench.flops_per_cell_update(3, 3) == 288
    assert bench.flops_per_cell_update(2, 2, dim=3, aniso=True) == 322


def test_flop_model_grows_with_the_problem():
    base = bench.flops_per_cell_update(2, 2)
    assert bench.flops_per_cell_update(3, 2) > base
    assert bench.flops_per_cell_update(2, 3) > base
    assert bench.flops_per_cell_update(2, 2, dim=3) > base
    assert bench.flops_per_cell_update(2, 2, aniso=True) > base


def test_roofline_records():
    r = bench.roofline(4.0e9, 1.0, traffic=2.5e9)  # 4 GB in 1 ms
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0)
    assert r["frac"] == pytest.approx(0.5)
    assert r["traffic"] == 2500000000
    a = bench.alu_roofline(39.3e9, 1.0, "f64")  # 39.3 GFLOP in 1 ms
    assert a["bound"] == "alu" and a["peak"] == 78.6
    assert a["achieved"] == pytest.approx(39.3)
    assert a["frac"] == pytest.approx(0.5)
    assert a["traffic"] is None
    assert bench.alu_roofline(1.0, 1.0, "f32")["peak"] == 157.3


def test_traffic_figures_hold_only_for_their_tile_steps_and_sources():
    for leg, t in bench.TRAFFIC.items():
        assert bench.traffic_of(leg, t["tile"], t["fuse"]) == t["bytes"], leg
        other = list(t["tile"])
        other[1] += 1
        assert bench.traffic_of(leg, other, t["fuse"]) is None
        assert bench.traffic_of(leg, t["tile"], 3 - t["fuse"]) is None
    assert bench.traffic_of("no such leg", [256, 31, 1], 2) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_bound_follows_the_max_rule():
    # 1 GB and 10 GFLOP per step in 0.2 ms: HBM ideal 0.125 ms > ALU ideal 0.127 ms? no:
    # FP64 peak 78.6 TFLOP/s -> 10e9 / 78.6e12 = 0.127 ms > 0.125 ms: the ALU bounds it
    r = bench.bound_record(1.0e9, 10.0e9, 0.2, "f64")
    assert r["bound"] == "alu"
    r = bench.bound_record(1.1e9, 10.0e9, 0.2, "f64", traffic=0.5e9, valu_insts=1.0e8, steps_per_launch=2)
    assert r["bound"] == "hbm"
    assert r["frac"] == pytest.approx(1.1e9 / 0.2e-3 / 8e12, rel=1e-3)
    # counter traffic per two-step launch of 0.4 ms; VALU issue 1e8 x 4 cycles / 1024 SIMDs / 2.4 GHz
    assert r["counter_frac"] == pytest.approx(0.5e9 / 0.4e-3 / 8e12, rel=1e-3)
    assert r["valu_issue_frac"] == pytest.approx(1.0e8 * 4 / 1024 / 2.4e9 / 0.4e-3, rel=1e-3)
    assert bench.bound_record(1.0e9, 1.0, 0.2, "f32")["counter_frac"] is None


def test_band_split_oracle_equals_the_full_step():
    """The CPU baseline's parallel row bands reproduce the oracle's full-grid steps bitwise."""
    import numpy as np

    from oracle import gp
    from paper_2404_01035_amd import inputs

    p, phi, mu = inputs.config_c2(precision="f64", n=(40, 37, 1))
    f, m = bench.oracle_band_steps(phi, mu, 3, 2, p, workers=3)
    rf, rm = gp.run(phi, mu, 3, 2, p)
    assert np.array_equal(f, rf) and np.array_equal(m, rm)


def test_valu_figures_hold_only_for_their_tile_steps_and_sources():
    for leg, t in bench.VALU.items():
        assert bench.valu_of(leg, t["tile"], t["fuse"]) == t["insts"], leg
        assert bench.valu_of(leg, t["tile"], 3 - t["fuse"]) is None
