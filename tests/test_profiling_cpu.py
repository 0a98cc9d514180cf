"""The rocprofv3 summary tool (paper_2505_13719_amd.profiling) on small
synthetic CSV files in the tool's column layout, each figure checked against
its hand-computed value: per-kernel trace statistics, the copy-calibrated HBM
bytes per launch the benchmark reads back (traffic_bytes_per_launch lines),
the L2 hit rate, and the derived CU memory-pipeline figures (L2 read latency,
reads in flight per CU by Little's law, TA busy share, TCP stall share)."""
import csv

import pytest

from paper_2505_13719_amd import profiling

KA = "void hl::k_a<double, 2>(hl::Tile const*)"
KB = "hl::k_b(int const*)"
COPY = "__amd_rocclr_copyBuffer"


def _trace_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for name, t0, t1 in rows:
            w.writerow([name, t0, t1])


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, cname, v) in enumerate(rows):
            w.writerow([i, name, cname, v])


def _table(out):
    """Rows of the first markdown table in out: kernel name -> cells."""
    rows = {}
    for line in out.splitlines():
        if line.startswith("| `"):
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            rows[cells[0].strip("`")] = cells[1:]
    return rows


def test_trace_statistics(tmp_path, capsys):
    p = tmp_path / "trace.csv"
    # k_a: 3 dispatches of 10, 20, 30 us; k_b: one of 40 us (times in ns)
    _trace_csv(p, [(KA, 0, 10_000), (KA, 50_000, 70_000), (KB, 100_000, 140_000), (KA, 200_000, 230_000)])
    profiling.trace(str(p))
    t = _table(capsys.readouterr().out)
    assert t[KA][:3] == ["3", "20.00", "0.1"]
    assert t[KB][:3] == ["1", "40.00", "0.0"]
    assert float(t[KA][3]) == pytest.approx(60.0)  # 60 of 100 us traced
    assert float(t[KB][3]) == pytest.approx(40.0)


def test_counters_copy_calibration(tmp_path, capsys):
    fe, wr = tmp_path / "fetch.csv", tmp_path / "write.csv"
    # the copy of 1024 KiB reads FETCH_SIZE 512 (factor 2) and writes 1024 (factor 1)
    _counter_csv(fe, [(COPY, "FETCH_SIZE", 512.0), (KA, "FETCH_SIZE", 100.0), (KA, "FETCH_SIZE", 300.0)])
    _counter_csv(wr, [(COPY, "WRITE_SIZE", 1024.0), (KA, "WRITE_SIZE", 10.0), (KA, "WRITE_SIZE", 30.0)])
    profiling.counters(str(fe), str(wr), copy_kib=1024)
    out = capsys.readouterr().out
    assert "FETCH_SIZE scaled by 2.0000, WRITE_SIZE by 1.0000" in out
    t = _table(out)
    assert t[KA][:3] == ["2", "200", "20"]
    # (200 KiB x 2 + 20 KiB x 1) x 1024 bytes per launch
    want = (200 * 2 + 20) * 1024
    line = next(x for x in out.splitlines() if x.startswith(f"traffic_bytes_per_launch[{KA}]"))
    assert line == f"traffic_bytes_per_launch[{KA}] = {want} dispatches=2"


def test_l2_hit_rate(tmp_path, capsys):
    p = tmp_path / "l2.csv"
    rows = []
    for name, hit, miss, rq in ((KA, 300.0, 100.0, 90.0), (KB, 10.0, 30.0, 30.0)):
        rows += [(name, "TCC_HIT_sum", hit), (name, "TCC_MISS_sum", miss), (name, "TCC_EA0_RDREQ_sum", rq),
                 (name, "TCC_EA0_RDREQ_32B_sum", 0.0)]
    _counter_csv(p, rows)
    profiling.l2(str(p))
    t = _table(capsys.readouterr().out)
    assert list(t) == [KA, KB]  # most misses first
    assert t[KA][3] == "0.750" and t[KB][3] == "0.250"
    assert t[KA][4] == "90"


def test_pmc_derived_figures(tmp_path, capsys):
    p = tmp_path / "pmc.csv"
    cyc = 1000.0  # per XCD; GRBM_GUI_ACTIVE sums the 8 XCDs
    rows = [(KA, "GRBM_GUI_ACTIVE", 8 * cyc), (KA, "TA_BUSY_avr", 600.0),
            (KA, "TCP_TCC_READ_REQ_sum", 2560.0), (KA, "TCP_TCC_READ_REQ_LATENCY_sum", 2560.0 * 400.0),
            (KA, "TCP_PENDING_STALL_CYCLES_sum", 256 * 0.5 * cyc),
            (KB, "GRBM_GUI_ACTIVE", 8 * 10.0), (KB, "TA_BUSY_avr", 1.0),
            (KB, "TCP_TCC_READ_REQ_sum", 1.0), (KB, "TCP_TCC_READ_REQ_LATENCY_sum", 100.0),
            (KB, "TCP_PENDING_STALL_CYCLES_sum", 0.0), (COPY, "GRBM_GUI_ACTIVE", 1e9)]
    _counter_csv(p, rows)
    profiling.pmc(str(p))
    out = capsys.readouterr().out
    header = next(x for x in out.splitlines() if x.startswith("| kernel"))
    cols = [c.strip() for c in header.strip().strip("|").split("|")][1:]
    t = _table(out)
    assert COPY not in t and list(t) == [KA, KB]  # this library's kernels, heaviest first
    a = dict(zip(cols, t[KA]))
    assert float(a["L2 read latency (cycles)"]) == pytest.approx(400.0)
    # Little's law: 2560 reads x 400 cycles over 256 CUs x 1000 cycles
    assert float(a["L2 reads in flight per CU"]) == pytest.approx(4.0)
    assert float(a["TA busy"]) == pytest.approx(0.6)
    assert float(a["TCP stalled on L2"]) == pytest.approx(0.5)
