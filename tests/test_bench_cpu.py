"""Host logic of bench.py (no GPU): the one-GPU contract, the issue-weighted
operation model behind the roofline entry, and the rule that the measured
HBM traffic is reported only for the kernel sources it was measured on."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_operation_model(bench):
    # per flight, per real collision, per ionisation, per polar/B flight
    assert (bench.OPS_PER_FLIGHT, bench.OPS_PER_REAL, bench.OPS_PER_ION,
            bench.OPS_PER_FLIGHT_POLAR_B) == (109, 163, 240, 200)
    c = {"n_real": 10, "n_null": 3, "n_masked": 1, "n_band": 2, "n_ion": 4}
    flights = 16  # every flight ends in a real, null or masked collision or a band cut
    assert bench.lane_ops(c) == flights * 109 + 10 * 163 + 4 * 240
    assert bench.lane_ops(c, polar_b=True) == flights * (109 + 200) + 10 * 163 + 4 * 240
    # the peak: 256 CUs x 4 SIMD16 x 16 lanes x 2.4 GHz
    assert bench.PEAK_LANE_OPS == pytest.approx(3.93216e13)


def test_traffic_only_for_the_measured_sources(bench, tmp_path, monkeypatch):
    t = {"fetch_kib_per_dispatch": 100.0, "write_kib_per_dispatch": 30.0,
         "fetch_scale": 2.0, "write_scale": 1.0, "kernel_source_sha256": bench.kernel_source_digest()}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() == (2.0 * 100.0 + 30.0) * 1024.0
    t["kernel_source_sha256"] = "0" * 64
    f.write_text(json.dumps(t))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic() is None


def test_digest_covers_the_kernel_and_its_build(bench):
    names = {os.path.basename(p) for p in bench.KERNEL_SOURCES}
    assert {"avm_kernels.hip", "avm_device.hpp", "avm_internal.hpp", "build.py"} <= names
    for p in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, p)), p
