"""Host-side logic of bench.py (no GPU): the counter summary that bench.py reads, the profile's validity check
and the vector-ALU roofline record."""
import csv
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

CHOSEN = "void tfsc::k_stat_wave<2, float, float, 2, false>(tfsc::StatArgs)"
FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(dirpath, rows):
    os.makedirs(dirpath, exist_ok=True)
    with open(os.path.join(dirpath, "c_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _row(disp, name, counter, value, t0=0, dur_ns=100_000_000):
    return {"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value,
            "Start_Timestamp": t0, "End_Timestamp": t0 + dur_ns}


def test_summarize_counters_medians_clock_and_calibrated_traffic(tmp_path, monkeypatch):
    prof = tmp_path / "counters.txt"
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    copy = "__amd_rocclr_copyBuffer"
    # pass 1: byte counters; the copy of 256 MiB reads 131072 KiB (factor 2) and writes 262144 KiB (factor 1)
    _write(tmp_path / "p_bytes", [
        _row(1, copy, "FETCH_SIZE", 131072.0), _row(1, copy, "WRITE_SIZE", 262144.0),
        # the first (cold) dispatch of the chosen kernel is left out of the medians
        _row(2, CHOSEN, "FETCH_SIZE", 9.0e9), _row(2, CHOSEN, "WRITE_SIZE", 9.0e9),
        _row(3, CHOSEN, "FETCH_SIZE", 1.0e6), _row(3, CHOSEN, "WRITE_SIZE", 2.0e3),
        _row(4, CHOSEN, "FETCH_SIZE", 3.0e6), _row(4, CHOSEN, "WRITE_SIZE", 2.0e3),
        _row(5, CHOSEN, "FETCH_SIZE", 2.0e6), _row(5, CHOSEN, "WRITE_SIZE", 2.0e3),
        # another kernel's counters are ignored
        _row(6, "void tfsc::k_stat_thread<2, float, float, 1, false>(tfsc::StatArgs)", "FETCH_SIZE", 7.0e9),
    ])
    # pass 2: instruction counters and the clock (GRBM_GUI_ACTIVE summed over 8 XCDs, 100 ms dispatches)
    sq = []
    for d in (2, 3, 4):
        sq += [_row(d, CHOSEN, "GRBM_GUI_ACTIVE", 8 * 2.0e8), _row(d, CHOSEN, "SQ_INSTS_VALU", 5.0e10),
               _row(d, CHOSEN, "SQ_INSTS_VALU_TRANS_F32", 4.0e9), _row(d, CHOSEN, "SQ_INSTS_VALU_TRANS_F64", 1.0e9),
               _row(d, CHOSEN, "SQ_INSTS_VALU_FMA_F32", 1.0e10), _row(d, CHOSEN, "SQ_INSTS_VALU_ADD_F64", 1.0e9)]
    _write(tmp_path / "p_sq", sq)
    bench.summarize_counters([str(tmp_path / "p_bytes"), str(tmp_path / "p_sq")], 1000020, "f32", "layer_ci",
                             "f0 bin, ln Mc", "4x4", 2.0, 1.0)
    rec = {}
    for line in prof.read_text().splitlines():
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    assert float(rec["FETCH_SIZE"]) == 2.0e6  # median of dispatches 3, 4, 5
    assert float(rec["WRITE_SIZE"]) == 2.0e3
    assert float(rec["clock_hz"]) == pytest.approx(2.0e9)  # 2e8 cycles per XCD in 0.1 s
    assert float(rec["valu_nontrans_insts"]) == pytest.approx(4.5e10)
    assert float(rec["fetch_factor"]) == pytest.approx(2.0) and float(rec["write_factor"]) == pytest.approx(1.0)
    assert float(rec["traffic_bytes"]) == pytest.approx(2.0e6 * 1024 * 2.0 + 2.0e3 * 1024 * 1.0)
    assert float(rec["flops"]) == pytest.approx(64 * (2 * 1.0e10 + 1.0e9 + 4.0e9 + 1.0e9))  # FMA x2, ADD, TRANS
    # the record is read back only for the same source, bank size, store, layout and order
    p = bench.measured_profile(1000020, "f32", "layer_ci", "f0 bin, ln Mc")
    assert p is not None and p["valu_insts"] == pytest.approx(5.0e10)
    assert bench.measured_profile(1000000, "f32", "layer_ci", "f0 bin, ln Mc") is None
    assert bench.measured_profile(1000020, "i16", "layer_ci", "f0 bin, ln Mc") is None
    assert bench.measured_profile(1000020, "f32", "layer_ci", "bank") is None
    text = prof.read_text().replace(rec["source_sha256"], "0" * 64)
    prof.write_text(text)
    assert bench.measured_profile(1000020, "f32", "layer_ci", "f0 bin, ln Mc") is None


def test_alu_roofline_against_the_rated_issue_rate():
    # 6.144e10 issue instructions in 0.1 s is the rated 614.4 G/s (1,024 SIMDs x 2.4 GHz / 4 cycles)
    prof = {"valu_insts": 7.0e10, "valu_nontrans_insts": 6.144e10, "clock_hz": 2.0e9, "flops": 7.864e12}
    r = bench.alu_roofline(prof, 0.1)
    assert r["bound"] == "alu" and r["peak"] == pytest.approx(614.4)
    assert r["achieved"] == pytest.approx(614.4) and r["frac"] == pytest.approx(1.0)
    # at the profile's own 2.0 GHz clock the same rate exceeds that clock's issue rate
    assert r["peak_at_profile_clock"] == pytest.approx(512.0) and r["frac_at_profile_clock"] == pytest.approx(1.2)
    assert r["flops"]["peak_tflops"] == pytest.approx(78.64, rel=1e-3) and r["flops"]["frac"] == pytest.approx(1.0, rel=1e-3)
    # the counter run's own fraction uses its dispatch time: 6.144e10 in 0.125 s at 2.0 GHz is 0.96
    r2 = bench.alu_roofline(dict(prof, dispatch_ns_counter_run=1.25e8), 0.1)
    assert r2["issue_in_profile_run"] == pytest.approx(0.96)
    assert "issue_in_profile_run" not in r
    # half the rate is half the rated peak; no profile gives no fraction
    assert bench.alu_roofline(prof, 0.2)["frac"] == pytest.approx(0.5)
    none = bench.alu_roofline(None, 0.1)
    assert none["frac"] is None and none["peak"] == pytest.approx(614.4)
