"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2505_13719_amd.profiling trace <kernel_trace.csv>
    python -m paper_2505_13719_amd.profiling counters <fetch counter_collection.csv> <write counter_collection.csv>
        [--copy-kib KIB]
    python -m paper_2505_13719_amd.profiling l2 <counter_collection.csv>
    python -m paper_2505_13719_amd.profiling pmc <counter_collection.csv> [--match TEXT]

`trace` prints, per kernel name, the dispatch count, average and total
duration and share of the traced kernel time (from rocprofv3
--kernel-trace CSV).  `counters` prints, per kernel, the average FETCH_SIZE
and WRITE_SIZE per dispatch (KiB, from two --pmc passes) and the HBM bytes
per launch after scaling each counter by what it reads for a plain device
copy of known size (the largest torch copy kernel in the same run moves
--copy-kib KiB each way, 1 GiB by default), plus one machine-readable line
per kernel: traffic_bytes_per_launch[<kernel>] = <bytes> dispatches=<n>.
`l2` prints, per kernel, the L2 (TCC) hits and misses per dispatch, the hit
rate and the read requests the L2 sends to memory (one --pmc pass with
TCC_HIT_sum, TCC_MISS_sum, TCC_EA0_RDREQ_sum and TCC_EA0_RDREQ_32B_sum).
`pmc` prints, for the kernels whose names contain TEXT (default: this
library's), every counter of the pass averaged per dispatch, and where the
pass holds them (GRBM_GUI_ACTIVE is summed over the 8 XCDs, so a dispatch's
clock count is GRBM_GUI_ACTIVE / 8; 256 CUs, one TA and one TCP each): the
TCP's mean L2 read latency (TCP_TCC_READ_REQ_LATENCY_sum /
TCP_TCC_READ_REQ_sum, cycles), the L2 reads in flight per CU on average
(TCP_TCC_READ_REQ_LATENCY_sum / (256 x cycles), Little's law), the TA's busy
share (TA_BUSY_avr / cycles) and the share of TCP cycles stalled on L2 data
(TCP_PENDING_STALL_CYCLES_sum / (256 x cycles)).
"""
import csv
import sys
from collections import defaultdict


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names)


def trace(path):
    by = defaultdict(list)
    for r in _rows(path):
        name = _col(r, "Kernel_Name", "KernelName", "Name")
        t0 = int(_col(r, "Start_Timestamp", "BeginNs", "Start"))
        t1 = int(_col(r, "End_Timestamp", "EndNs", "End"))
        by[name].append((t1 - t0) * 1e-3)
    total = sum(sum(v) for v in by.values())
    print("| kernel | calls | avg us | total ms | % |")
    print("|---|---:|---:|---:|---:|")
    for name, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        print(f"| `{name}` | {len(v)} | {sum(v) / len(v):.2f} | {sum(v) * 1e-3:.1f} | {100 * sum(v) / total:.2f} |")


def _counter(path, cname):
    acc = defaultdict(lambda: [0.0, 0])
    for r in _rows(path):
        if _col(r, "Counter_Name", "CounterName") != cname:
            continue
        name = _col(r, "Kernel_Name", "KernelName")
        acc[name][0] += float(_col(r, "Counter_Value", "CounterValue"))
        acc[name][1] += 1
    return {k: (s / n, n) for k, (s, n) in acc.items()}


def _max_copy(path, cname):
    """Largest single dispatch of a runtime copy kernel (the calibration
    copy: the bench's 1 GiB device-to-device copy)."""
    best, name = 0.0, None
    for r in _rows(path):
        k = _col(r, "Kernel_Name", "KernelName")
        if _col(r, "Counter_Name", "CounterName") == cname and "hl::" not in k and "copy" in k.lower():
            v = float(_col(r, "Counter_Value", "CounterValue"))
            if v > best:
                best, name = v, k
    return best, name


def counters(fetch_path, write_path, copy_kib=1 << 20):
    fe = _counter(fetch_path, "FETCH_SIZE")
    wr = _counter(write_path, "WRITE_SIZE")
    cf, cal = _max_copy(fetch_path, "FETCH_SIZE")
    cw, _ = _max_copy(write_path, "WRITE_SIZE")
    fs = copy_kib / cf if cf > 0 else 1.0
    ws = copy_kib / cw if cw > 0 else 1.0
    print(f"Calibration: the largest `{cal}` dispatch (a {copy_kib} KiB device copy) reads FETCH_SIZE = "
          f"{cf:.0f} KiB and WRITE_SIZE = {cw:.0f} KiB: FETCH_SIZE scaled by {fs:.4f}, WRITE_SIZE by {ws:.4f}.\n"
          if cal else "No copy dispatch found: counters unscaled.\n")
    print("| kernel | dispatches | FETCH KiB | WRITE KiB | HBM MB / launch (scaled) |")
    print("|---|---:|---:|---:|---:|")
    lines = []
    for name, (f, n) in sorted(fe.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        w = wr.get(name, (0.0, 0))[0]
        b = (f * fs + w * ws) * 1024
        print(f"| `{name}` | {n} | {f:.0f} | {w:.0f} | {b / 1e6:.1f} |")
        lines.append(f"traffic_bytes_per_launch[{name}] = {b:.0f} dispatches={n}")
    print()
    print("\n".join(lines))


def l2(path, top=12):
    c = {k: _counter(path, k) for k in ("TCC_HIT_sum", "TCC_MISS_sum", "TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum")}
    names = sorted(c["TCC_MISS_sum"], key=lambda k: -c["TCC_MISS_sum"][k][0] * c["TCC_MISS_sum"][k][1])
    print("| kernel | dispatches | L2 hits / launch | L2 misses / launch | hit rate | memory read requests / launch "
          "| of them 32 B |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for name in names[:top]:
        h, n = c["TCC_HIT_sum"].get(name, (0.0, 0))
        m = c["TCC_MISS_sum"][name][0]
        rq = c["TCC_EA0_RDREQ_sum"].get(name, (0.0, 0))[0]
        r32 = c["TCC_EA0_RDREQ_32B_sum"].get(name, (0.0, 0))[0]
        rate = h / (h + m) if h + m > 0 else 0.0
        print(f"| `{name}` | {n} | {h:.4g} | {m:.4g} | {rate:.3f} | {rq:.4g} | {r32:.4g} |")


def pmc(path, match="hl::", top=12, cus=256, xcds=8):
    names = []
    for r in _rows(path):
        c = _col(r, "Counter_Name", "CounterName")
        if c not in names:
            names.append(c)
    c = {k: _counter(path, k) for k in names}
    kern = {k for v in c.values() for k in v if match in k}
    # heaviest first: by busy cycles over all dispatches when the pass holds
    # them, else by the counter with the largest total
    tot = {x: sum(v[0] * v[1] for v in c[x].values()) for x in names}
    first = "GRBM_GUI_ACTIVE" if "GRBM_GUI_ACTIVE" in c else max(names, key=lambda x: tot[x])
    order = sorted(kern, key=lambda k: -c[first].get(k, (0.0, 0))[0] * c[first].get(k, (0.0, 0))[1])[:top]
    derived = []
    cyc = lambda k: max(c["GRBM_GUI_ACTIVE"][k][0] / xcds, 1.0)  # noqa: E731
    if "TCP_TCC_READ_REQ_LATENCY_sum" in c and "TCP_TCC_READ_REQ_sum" in c:
        derived.append(("L2 read latency (cycles)", lambda k: c["TCP_TCC_READ_REQ_LATENCY_sum"][k][0] /
                        max(c["TCP_TCC_READ_REQ_sum"][k][0], 1.0)))
        if "GRBM_GUI_ACTIVE" in c:
            derived.append(("L2 reads in flight per CU",
                            lambda k: c["TCP_TCC_READ_REQ_LATENCY_sum"][k][0] / (cus * cyc(k))))
    if "TA_BUSY_avr" in c and "GRBM_GUI_ACTIVE" in c:
        derived.append(("TA busy", lambda k: c["TA_BUSY_avr"][k][0] / cyc(k)))
    if "TCP_PENDING_STALL_CYCLES_sum" in c and "GRBM_GUI_ACTIVE" in c:
        derived.append(("TCP stalled on L2", lambda k: c["TCP_PENDING_STALL_CYCLES_sum"][k][0] / (cus * cyc(k))))
    names = sorted(names)
    print("| kernel | dispatches | " + " | ".join(names + [d[0] for d in derived]) + " |")
    print("|---|---:|" + "---:|" * (len(names) + len(derived)))
    for k in order:
        n = c[first].get(k, (0.0, 0))[1]
        vals = [f"{c[x].get(k, (0.0, 0))[0]:.4g}" for x in names]
        der = []
        for _, f in derived:
            try:
                der.append(f"{f(k):.3g}")
            except KeyError:
                der.append("-")
        print(f"| `{k}` | {n} | " + " | ".join(vals + der) + " |")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2])
    elif sys.argv[1] == "l2":
        l2(sys.argv[2])
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[sys.argv.index("--match") + 1] if "--match" in sys.argv else "hl::")
    else:
        kib = 1 << 20
        if "--copy-kib" in sys.argv:
            kib = int(sys.argv[sys.argv.index("--copy-kib") + 1])
        counters(sys.argv[2], sys.argv[3], kib)
