"""Host logic of bench.py: shear-variant arguments and the lookup of measured
HBM traffic (per shear of the step, per variant, only on the kernel source the
counters were taken on)."""
import argparse
import json

import pytest

import bench


def test_variant_arguments():
    assert bench.parse_variant("7") == 7
    assert bench.parse_variant("2,0,10") == (2, 0, 10)
    with pytest.raises(argparse.ArgumentTypeError):
        bench.parse_variant("1,2")
    assert bench.variant_key(3) == "3,3,3"
    assert bench.variant_key((2, 0, 10)) == "2,0,10"
    assert bench.variant_key([1, 1, 4]) == "1,1,4"


def fake_profiles(tmp_path, monkeypatch, hash_=None, workload="w"):
    (tmp_path / "profiles").mkdir()
    d = {"storage": "f64", "workload": workload,
         "kernel_source_hash": hash_ if hash_ is not None else bench.kernel_source_hash(),
         "hbm_bytes_per_launch_by_shear": {"2": [30.0, 20.0, 10.0], "10": [31.0, 21.0, 13.0]}}
    (tmp_path / "profiles" / "shear_traffic_f64.json").write_text(json.dumps(d))
    real = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: real)


def test_traffic_is_the_mean_over_the_three_shears(tmp_path, monkeypatch):
    fake_profiles(tmp_path, monkeypatch)
    assert bench.measured_traffic("f64", 2, "w") == pytest.approx(20.0)
    assert bench.measured_traffic("f64", (2, 2, 10), "w") == pytest.approx((30.0 + 20.0 + 13.0) / 3)
    assert bench.measured_traffic("f64", (10, 2, 2), "w") == pytest.approx((31.0 + 20.0 + 10.0) / 3)


def test_traffic_is_null_when_unprofiled_or_stale(tmp_path, monkeypatch):
    fake_profiles(tmp_path, monkeypatch)
    assert bench.measured_traffic("f64", (2, 3, 2), "w") is None      # variant 3 not profiled
    assert bench.measured_traffic("f64", 2, "other") is None          # other workload
    assert bench.measured_traffic("f32", 2, "w") is None              # no file


def test_traffic_is_null_after_a_kernel_change(tmp_path, monkeypatch):
    fake_profiles(tmp_path, monkeypatch, hash_="0" * 16)
    assert bench.measured_traffic("f64", 2, "w") is None


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr
