"""Host-side arithmetic of bench.py, the code behind every reported figure
(no GPU): the refusal of more than one GPU, the barotropic words per step
against a count by hand, the rooflines from stage times, and the three
summaries of rocprofv3 output (traffic scaled by the copy calibration, SQ
counters split by precision, kernel-trace table) on small synthetic files.
"""
import csv
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2309_06662_amd import inputs  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_barotropic_words_against_a_count_by_hand():
    # Ns = 60: M = 90 substeps, 7 per launch -> launches at m0 = 0, 7, ..., 84
    # (13, the last of 6). The window's first nonzero weight is substep 31.
    # Reads per column: 5.5 words in every launch (eta, U, V, G_U, G_V and a
    # 4-byte wet count), the two transport sums in the 12 launches after the
    # first, the three window sums in the 8 launches starting at m0 >= 35:
    # 71.5 + 24 + 24 = 119.5. Writes: 6 in the last launch (eta, U, V and the
    # three means); 5 in the other 12 (eta, U, V, two transport sums) plus the
    # three window sums in the 8 that reach substep 31 (m0 = 28 ... 77):
    # 6 + 60 + 24 = 90. An odd launch count adds the copy back of eta, U, V
    # (3 read, 3 written): 119.5 + 90 + 6 = 215.5.
    words, launches = bench.baro_words_per_step(60, fuse=7)
    assert launches == 13
    assert words == 215.5
    # an even launch count has no copy back: M = 45, 7 per launch -> 7 launches
    assert bench.baro_words_per_step(30, fuse=7)[1] == 7


def test_rooflines_from_stage_times(monkeypatch):
    monkeypatch.setattr(bench, "_traffic_from_profiles", lambda *a, **k: None)
    w = inputs.LATLON_TWELFTH
    cells = 4320 * 1800 * 100
    main, other, stages = bench.roofline(w, "fp32", {"tendency": 20.0, "barotropic": 4.0, "column": 4.0}, 13)
    # 12 words of 4 bytes per cell in 20 ms
    assert main["bound"] == "hbm" and main["kernel"] == "k_tend"
    assert main["achieved"] == pytest.approx(12 * 4 * cells / 0.020 / 1e9, abs=0.05)
    assert main["frac"] == pytest.approx(main["achieved"] / 8000.0, abs=1e-4)
    assert other["bound"] == "alu" and other["frac"] < main["frac"]
    # column: 6 words per cell in 4 ms; barotropic: 215.5 FP64 words per column in 4 ms
    assert stages["column"]["achieved"] == pytest.approx(6 * 4 * cells / 0.004 / 1e9, abs=0.05)
    assert stages["barotropic"]["bytes_per_step"] == 215.5 * 8 * 4320 * 1800
    assert stages["barotropic"]["share_of_step"] == pytest.approx(4.0 / 28.0, abs=1e-4)
    # FP64 doubles the bytes of the same times
    main64, _, _ = bench.roofline(w, "fp64", {"tendency": 20.0, "barotropic": 4.0, "column": 4.0}, 13)
    assert main64["achieved"] == pytest.approx(2 * main["achieved"], abs=0.1)


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        wr.writeheader()
        for d, name, counter, value in rows:
            wr.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_record_scales_by_the_copy(tmp_path):
    gib = 1 << 30
    # the copy reads and writes 1 GiB; its FETCH_SIZE reads half of that (KiB), WRITE_SIZE all of it
    _counter_csv(tmp_path / "cf.csv", [(1, "copy_kernel", "FETCH_SIZE", gib / 2048)])
    _counter_csv(tmp_path / "cw.csv", [(1, "copy_kernel", "WRITE_SIZE", gib / 1024)])
    # two dispatches of the kernel, counters split over two rows each (summed per dispatch)
    _counter_csv(tmp_path / "kf.csv", [(5, "k_tend<float>", "FETCH_SIZE", 600.0), (5, "k_tend<float>", "FETCH_SIZE", 400.0),
                                       (9, "k_tend<float>", "FETCH_SIZE", 3000.0), (7, "other", "FETCH_SIZE", 1e9)])
    _counter_csv(tmp_path / "kw.csv", [(5, "k_tend<float>", "WRITE_SIZE", 500.0), (9, "k_tend<float>", "WRITE_SIZE", 1500.0)])
    out = tmp_path / "rec.json"
    a = SimpleNamespace(copy_fetch=str(tmp_path / "cf.csv"), copy_write=str(tmp_path / "cw.csv"),
                        fetch=str(tmp_path / "kf.csv"), write=str(tmp_path / "kw.csv"), name="k_tend<float",
                        kernel="k_tend", steady=2, copy_bytes=float(gib), workload="w", precision="fp32",
                        command=["c"], out=str(out))
    bench.pmc_summary(a)
    rec = json.load(open(out))
    assert rec["fetch_kib_per_dispatch"] == [1000.0, 3000.0]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    # mean of the two steady dispatches: (1000 + 3000) / 2 KiB fetched x 2, (500 + 1500) / 2 KiB written
    assert rec["hbm_fetch_bytes_per_launch"] == pytest.approx(2000 * 1024 * 2.0)
    assert rec["hbm_write_bytes_per_launch"] == pytest.approx(1000 * 1024 * 1.0)
    assert rec["source_sha256_16"] == bench._src_hash(bench._kernel_src("k_tend"))


def test_sq_summary_splits_precisions_and_takes_full_launches(tmp_path):
    names = {1: "void ocn::k_tend<float, 32, 16, false, false>(ocn::DevState, int, int)",
             2: "void ocn::k_baro_fused<64, 24, 7>(ocn::DevState, double, int)",
             3: "void ocn::k_baro_fused<64, 24, 6>(ocn::DevState, double, int)",
             4: "void ocn::k_column<float, 100>(ocn::DevState)",
             5: "void ocn::k_tend<double, 16, 16, false, false>(ocn::DevState, int, int)",
             6: "void ocn::k_baro_fused<64, 24, 7>(ocn::DevState, double, int)",
             7: "void ocn::k_column<double, 100>(ocn::DevState)"}
    first = [("SQ_INSTS_VALU", 1e9), ("SQ_INSTS_LDS", 1e8), ("SQ_INSTS_SALU", 5e8), ("SQ_WAVES", 100.0)]
    second = [("GRBM_GUI_ACTIVE", 8e7), ("SQ_LDS_BANK_CONFLICT", 1.0), ("SQ_LDS_IDX_ACTIVE", 10.0)]
    _counter_csv(tmp_path / "a.csv", [(d, n, c, v * d) for d, n in names.items() for c, v in first])
    _counter_csv(tmp_path / "b.csv", [(d, n, c, v) for d, n in names.items() for c, v in second])
    for prec, tend, baro, col in (("fp32", 1, 2, 4), ("fp64", 5, 6, 7)):
        out = tmp_path / f"sq_{prec}.txt"
        a = SimpleNamespace(sq1=str(tmp_path / "a.csv"), sq2=str(tmp_path / "b.csv"), precision=prec,
                            workload=inputs.LATLON_TWELFTH.name, command=["c"], out=str(out))
        bench.sq_summary(a)
        text = out.read_text()
        assert f"(dispatch {tend}/{tend})" in text and f"(dispatch {baro}/{baro})" in text
        assert f"(dispatch {col}/{col})" in text and "<64, 24, 6>" not in text
        # VALU busy = instructions x 4 cycles / (1024 SIMDs x GUI cycles / 8 XCDs)
        busy = 1e9 * tend * 4 / (1024 * 8e7 / 8)
        assert f"VALU busy {busy:.2f}" in text
        # per cell: instructions x 64 lanes / cells
        assert f"VALU lane-instructions per cell: {1e9 * tend * 64 / (4320 * 1800 * 100):.0f}" in text


def test_stats_summary_table_and_tendency_launches(tmp_path):
    d = tmp_path / "stats"
    d.mkdir()
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        wr = csv.writer(f)
        wr.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        wr.writerow(["void ocn::k_tend<float, 32, 16, false, false>(ocn::DevState, int, int)", 3, 60e6, 20e6, 90.0,
                     16e6, 22e6, 1.0])
    with open(d / "run_kernel_trace.csv", "w", newline="") as f:
        wr = csv.writer(f)
        wr.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for i, us in enumerate((16000.0, 22000.0, 21000.0)):
            wr.writerow([i + 1, "void ocn::k_tend<float, 32, 16, false, false>(ocn::DevState, int, int)",
                         1000000 * i, 1000000 * i + int(us * 1000)])
    out = tmp_path / "st.txt"
    bench.stats_summary(SimpleNamespace(stats_dir=str(d), workload="w", command=["c"], out=str(out)))
    text = out.read_text()
    assert "20000.0" in text and "60000.0" in text
    # the first launch is the start step; the steady mean is over the others
    assert "16000.0, 22000.0, 21000.0; steady (AB2) mean 21500.0 us" in text


def test_valu_issue_view_reads_the_summary_of_the_current_source(tmp_path):
    cur = bench._src_hash(bench._kernel_src("k_tend"))
    body = ("void ocn::k_tend<float, 32, 16, false, false> (dispatch 5/5): 1 cycles per XCD\n"
            "  VALU lane-instructions per cell: 800; LDS per cell: 90.0; SALU/VALU 0.35\n")
    good, stale = tmp_path / "good.txt", tmp_path / "stale.txt"
    good.write_text(f"# source sha256/16 of k_tend.hip: {cur}\n" + body)
    stale.write_text("# source sha256/16 of k_tend.hip: 0000000000000000\n" + body)
    w = inputs.LATLON_TWELFTH
    assert bench._valu_per_cell_from_profiles(w.name, "fp32", path=str(good)) == 800.0
    assert bench._valu_per_cell_from_profiles(w.name, "fp32", path=str(stale)) is None
    # 800 instructions x 7.776e8 cells in 20 ms against 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    v = bench.valu_issue_view(w, "fp32", {"tendency": 20.0}, per_cell=800.0)
    rate = 800.0 * 4320 * 1800 * 100 / 0.020
    assert v["achieved"] == pytest.approx(rate / 1e12, abs=0.01)
    assert v["frac"] == pytest.approx(rate / (256 * 4 * 16 * 2.4e9), abs=1e-4)
