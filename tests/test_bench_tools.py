"""The measurement helpers of bench.py on synthetic rocprofv3 CSV files: the
kernel-time and counter tables average working dispatches only (launches
queued after a block's stop return at once), and the traffic record scales
FETCH_SIZE / WRITE_SIZE by the copy calibration.  CPU only."""
import csv
import io
import json
import os
import sys
from contextlib import redirect_stdout

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

KNAME = "void (anonymous namespace)::k_dslash_sr<float, false, true>((anonymous namespace)::DslashArgs<float>)"


def _write(path, rows, fields):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _trace(tmp_path):
    rows, t = [], 0
    # 6 working dispatches of 1000..1005 us and 3 no-op ones of 20 us
    for k, dur in enumerate([1000, 1001, 1002, 20, 1003, 20, 1004, 1005, 20]):
        rows.append({"Kernel_Name": KNAME, "Grid_Size_X": 16777216, "Start_Timestamp": t,
                     "End_Timestamp": t + dur * 1000})
        t += dur * 1000 + 5000
    rows.append({"Kernel_Name": "k_reduce", "Grid_Size_X": 6144, "Start_Timestamp": t, "End_Timestamp": t + 7000})
    _write(str(tmp_path / "stats" / "run_kernel_trace.csv"), rows,
           ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"])


def _counters(path, name, kernel, grid, values_durs):
    rows, t = [], 0
    for i, (v, dur) in enumerate(values_durs):
        rows.append({"Dispatch_Id": i, "Kernel_Name": kernel, "Grid_Size": grid, "Counter_Name": name,
                     "Counter_Value": v, "Start_Timestamp": t, "End_Timestamp": t + dur * 1000})
        t += dur * 1000 + 1000
    _write(path, rows, ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value",
                        "Start_Timestamp", "End_Timestamp"])


def test_kernel_table_averages_working_dispatches(tmp_path):
    _trace(tmp_path)
    buf = io.StringIO()
    with redirect_stdout(buf):
        bench.summarize_profile(str(tmp_path / "stats"), [], "k_dslash")
    line = [ln for ln in buf.getvalue().splitlines() if "k_dslash_sr" in ln][0]
    cells = [c.strip() for c in line.strip("|").split("|")]
    assert cells[0] == "`k_dslash_sr<float, false, true>`"
    assert cells[2] == "9" and cells[3] == "6"         # dispatches, working
    assert float(cells[4]) == pytest.approx(1002.5)     # mean of the working ones only
    assert float(cells[5]) == 1000.0 and float(cells[6]) == 1005.0


def test_counter_table_drops_noop_dispatches(tmp_path):
    _trace(tmp_path)
    _counters(str(tmp_path / "fetch" / "run_counter_collection.csv"), "FETCH_SIZE", KNAME, 16777216,
              [(100.0, 1000), (102.0, 1002), (1.0, 20), (104.0, 1004)])
    buf = io.StringIO()
    with redirect_stdout(buf):
        bench.summarize_profile(str(tmp_path / "stats"), [str(tmp_path / "fetch")], "k_dslash")
    line = [ln for ln in buf.getvalue().splitlines() if "k_dslash_sr" in ln and "FETCH" not in ln][-1]
    cells = [c.strip() for c in line.strip("|").split("|")]
    assert cells[2] == "3" and float(cells[3]) == pytest.approx(102.0)


def test_traffic_record_scales_by_copy_calibration(tmp_path):
    _counters(str(tmp_path / "f" / "run_counter_collection.csv"), "FETCH_SIZE", KNAME, 16777216,
              [(1000.0, 1000), (1.0, 20), (1000.0, 1000)])
    _counters(str(tmp_path / "w" / "run_counter_collection.csv"), "WRITE_SIZE", KNAME, 16777216,
              [(500.0, 1000), (0.0, 20), (500.0, 1000)])
    # the 256 MiB copy reads half its bytes in FETCH_SIZE units and all of them in WRITE_SIZE units
    _counters(str(tmp_path / "cf" / "run_counter_collection.csv"), "FETCH_SIZE", "__amd_rocclr_copyBuffer", 1,
              [(131072.0, 50)])
    _counters(str(tmp_path / "cw" / "run_counter_collection.csv"), "WRITE_SIZE", "__amd_rocclr_copyBuffer", 1,
              [(262144.0, 50)])
    buf = io.StringIO()
    with redirect_stdout(buf):
        bench.traffic_record("k_dslash_sr<float, false, true>", "test", str(tmp_path / "f"), str(tmp_path / "w"),
                             str(tmp_path / "cf"), str(tmp_path / "cw"), grid=16777216)
    rec = json.loads(buf.getvalue())
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    assert rec["dispatches"] == 2
    assert rec["traffic_bytes_per_launch"] == pytest.approx((1000.0 * 2.0 + 500.0) * 1024)


def test_schur_bytes_count_half_lattice_passes_once():
    """Five passes over a compact block of V/2 sites x 12 complex x L columns
    are 5 x 12 L reals per site of the whole lattice."""
    L, s = 8, 4
    V = 16
    links = 2 * 4 * V * 18          # two launches, every link once
    clover = V * 72                 # half the sites' blocks in each of the two launches
    spinors = 5 * (V // 2) * 12 * 2 * L
    assert bench.schur_bytes_per_site(L, s) * V == (links + clover + spinors) * s


def test_operator_bytes_per_site():
    assert bench.dslash_bytes_per_site(8, 4) == (4 * 18 + 72 + 48 * 8) * 4
    assert bench.dslash_bytes_per_site(8, 4, 12) == (4 * 12 + 72 + 48 * 8) * 4


def test_evenodd_figures_price_the_gram_launch(monkeypatch):
    """The even-odd leg prices the plain Schur applications and, when the
    frame's Grams ride in the second Schur launch, that launch with one extra
    compact pass over R~ (12 L reals per site of the whole lattice)."""
    L, V = 8, 4096
    info = {"main_width": L, "dslash_calls_fp32_main": 100, "dslash_ms_fp32_main": 100 * 2.0,
            "update_calls_main": [100, 100, 50], "update_ms_main": [1.0, 1.0, 50 * 2.5],
            "iterations": 50, "true_residual_max": 1e-13, "gram_operator": 1}

    class _Lat:
        def make_opts(self, **kw):
            return kw

    monkeypatch.setattr(bench, "timed_solves", lambda *a, **k: ([info], 2.0))
    out = bench.evenodd_figures(_Lat(), None, None, 64, V, 1, 0, "t", 1.0)
    plain = V * bench.schur_bytes_per_site(L, 4)
    assert out["schur_operator"]["bytes_per_application"] == plain
    assert out["schur_operator"]["avg_application_us"] == pytest.approx(2000.0)
    g = out["schur_gram_launch"]
    assert g["bytes_per_launch"] == plain + V * 12 * L * 4
    assert g["avg_launch_us"] == pytest.approx(2500.0) and g["launches_timed"] == 50
    info["gram_operator"] = 0
    assert "schur_gram_launch" not in bench.evenodd_figures(_Lat(), None, None, 64, V, 1, 0, "t", 1.0)
