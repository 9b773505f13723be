"""Host logic of bench.py (no GPU): the one-GPU guard, the HBM-traffic summary written from rocprofv3
counter CSVs, the stale-summary rule and the median of the timed repetitions."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_step_byte_model():
    class Plan:
        x_fused = False

    assert bench.step_passes_hbm(Plan(), 300) == 12.0
    Plan.x_fused = True
    assert bench.step_passes_hbm(Plan(), 1) == 12.0  # one step: x r2c and x c2r, no fused pass
    assert bench.step_passes_hbm(Plan(), 300) == pytest.approx(10.0 + 2.0 / 300)


def test_median_spread():
    assert bench.median_spread([3.0, 1.0, 2.0, 5.0, 4.0]) == (3.0, 1.0, 5.0)


def test_write_traffic_calibration_and_kernel_names(tmp_path):
    """Counters in 2 KiB (fetch) and 1 KiB (write) units, as on MI355X: the 1 GiB copy reads 2^19 and
    writes 2^20 units.  The step kernels' names carry nested template arguments (Spread<...>); the
    state set-up's y pass (one dispatch) must not replace the step's (four dispatches)."""
    n = 64
    rb = n**3 * 4
    z = "void pfc::last_axis_kernel<float, pfc::Spread<pfc::Radices<16, 8, 16, 0>, 32>, 16, 0, 1, false, 2, true, 2>(x)"
    z_other_mode = "void pfc::last_axis_kernel<float, pfc::Radices<2, 16, 16, 0>, 16, 2, 1, true, 2, true, 1>(x)"
    xr = "void pfc::x_r2c_kernel<float, pfc::Radices<16, 16, 1, 0>, 16, true, false, true>(x)"
    xr_plain = "void pfc::x_r2c_kernel<float, pfc::Radices<16, 16, 1, 0>, 16, false, false, true>(x)"
    xc = "void pfc::x_c2r_kernel<float, pfc::Radices<8, 4, 8, 0>, 2, 0, false, false, true>(x)"
    y_step = "void pfc::axis_c2c_kernel<float, pfc::Radices<16, 2, 16, 0>, 8, -1, 1, false, 1>(x)"
    y_init = "void pfc::axis_c2c_kernel<float, pfc::Radices<16, 2, 16, 0>, 16, -1, 1, false, 1>(x)"
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(x)>(x)"
    fu, wu = 2048.0, 1024.0
    fetch = [(copy, 2**30 / fu)] * 3 + [(y_init, 9 * rb / fu)] + [(y_step, 1.05 * rb / fu)] * 4 + \
            [(z, 2.06 * rb / fu)] * 3 + [(z_other_mode, 7 * rb / fu)] + [(xr, rb / fu)] * 3 + \
            [(xr_plain, 5 * rb / fu)] + [(xc, rb / fu)] * 3
    write = [(copy, 2**30 / wu)] * 3 + [(y_init, 9 * rb / wu)] + [(y_step, rb / wu)] * 4 + \
            [(z, 2.0 * rb / wu)] * 3 + [(z_other_mode, 7 * rb / wu)] + [(xr, rb / wu)] * 3 + \
            [(xr_plain, 5 * rb / wu)] + [(xc, rb / wu)] * 3
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", write)
    out = str(tmp_path / "traffic.txt")
    bench.write_traffic(str(tmp_path / "f"), str(tmp_path / "w"), out, "cmd", n)
    t = json.load(open(out))
    assert t["kernel_hash"] == bench.kernel_hash() and t["grid"] == [n, n, n]
    assert t["fetch_factor_bytes_per_unit"] == pytest.approx(fu) and t["write_factor_bytes_per_unit"] == pytest.approx(wu)
    k = t["kernels"]
    assert set(k) == {"y_fwd_or_inv", "z_fused_update", "x_r2c_cube", "x_c2r"}
    assert k["y_fwd_or_inv"]["dispatches"] == 4 and k["y_fwd_or_inv"]["traffic_over_alg"] == pytest.approx(1.025, abs=1e-3)
    assert k["z_fused_update"]["dispatches"] == 3 and "Spread" in k["z_fused_update"]["kernel"]
    assert k["z_fused_update"]["traffic_over_alg"] == pytest.approx(1.015, abs=1e-3)
    assert k["x_r2c_cube"]["traffic_over_alg"] == pytest.approx(1.0, abs=1e-3)
    assert k["x_c2r"]["alg_bytes_per_launch"] == 2 * rb


def test_traffic_is_null_when_the_kernels_changed(tmp_path, monkeypatch):
    good = {"kernel_hash": bench.kernel_hash(), "kernels": {"z_fused_update": {"hbm_bytes_per_launch": 123}}}
    stale = dict(good, kernel_hash="0" * 16)
    p = tmp_path / "t.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    p.write_text(json.dumps(good))
    assert bench.measured_traffic("z_fused_update") == 123
    assert bench.measured_traffic("x_c2r") is None
    p.write_text(json.dumps(stale))
    assert bench.measured_traffic("z_fused_update") is None
