"""Reduce rocprofv3 CSV output to short text summaries.

    python -m paper_2204_10822_amd.profsum stats  <kernel_stats.csv>  [top]
    python -m paper_2204_10822_amd.profsum counter <counter_collection.csv> <COUNTER>
    python -m paper_2204_10822_amd.profsum grids <kernel_trace.csv> [top]
    python -m paper_2204_10822_amd.profsum requests <read_counters.csv> <write_counters.csv> [top]

`stats` prints the top kernels by summed duration.  `counter` prints, per kernel
name, the dispatch count and the mean value of one counter per dispatch (for
FETCH_SIZE / WRITE_SIZE this is KiB per dispatch), plus the values seen for the
device copy kernels used as a calibration of known size.  `grids` splits the
kernel time by (kernel, grid size): on the AMG hierarchy the grid size names the
level.  `requests` combines a pass of the size-split L2->memory read-request
counters (TCC_EA0_RDREQ_sum and its _32B/_64B/_128B parts) with one of the write
requests (TCC_EA0_WRREQ_sum, TCC_EA0_WRREQ_64B_sum; the others carry 32 B) into
bytes per dispatch: HBM traffic counted request by request at its own size.
"""
from __future__ import annotations

import collections
import csv
import re
import sys


def _demangle_vp(name: str) -> str:
    """Readable name for a mangled vp:: kernel template the profiler left mangled
    (its demangler does not know _Float16, mangled DF16_)."""
    m = re.match(r"_ZN2vp(?:3net)?(\d+)", name)
    if not m:
        return name
    k = m.end()
    ln = int(m.group(1))
    ident = name[k:k + ln]
    k += ln
    if k >= len(name) or name[k] != "I":
        return ident
    k += 1
    args = []
    while k < len(name) and name[k] != "E":
        if name.startswith("Li", k):
            e = name.index("E", k)
            args.append(name[k + 2:e])
            k = e + 1
        elif name.startswith("Lb", k):
            args.append("true" if name[k + 2] == "1" else "false")
            k = name.index("E", k) + 1
        elif name.startswith("DF16_", k):
            args.append("_Float16")
            k += 5
        elif name[k] in "fdi":
            args.append({"f": "float", "d": "double", "i": "int"}[name[k]])
            k += 1
        elif name[k].isdigit():
            mm = re.match(r"\d+", name[k:])
            n = int(mm.group(0))
            k += len(mm.group(0))
            args.append(name[k:k + n])
            k += n
        else:
            return ident + "<?>"
    return f"{ident}<{', '.join(args)}>"


def _short(name: str) -> str:
    if name.startswith("_Z"):
        return _demangle_vp(name)
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*$", "", name)           # drop the argument list
    name = name.replace("void ", "").replace("vp::", "")
    return name


def stats(path: str, top: int = 25) -> None:
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print(f"{'kernel':58s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}")
    for r in rows[:top]:
        t = float(r["TotalDurationNs"])
        print(f"{_short(r['Name'])[:58]:58s} {int(r['Calls']):7d} {t / 1e6:10.3f} "
              f"{float(r['AverageNs']) / 1e3:10.2f} {100 * t / tot:6.2f}")
    print(f"total kernel time {tot / 1e6:.3f} ms over {sum(int(r['Calls']) for r in rows)} dispatches")


def counter(path: str, cname: str) -> None:
    acc = collections.defaultdict(list)
    grids = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != cname:
            continue
        k = _short(r["Kernel_Name"])
        acc[k].append(float(r["Counter_Value"]))
        grids[k] = r.get("Grid_Size", "")
    print(f"{cname}: mean per dispatch (KiB for FETCH_SIZE/WRITE_SIZE)")
    print(f"{'kernel':58s} {'n':>5s} {'mean':>14s} {'grid':>10s}")
    for k, v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        print(f"{k[:58]:58s} {len(v):5d} {sum(v) / len(v):14.1f} {grids[k]:>10s}")


def _means(path: str) -> tuple[dict, dict, dict]:
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    grid = {}
    for r in csv.DictReader(open(path)):
        k = _short(r["Kernel_Name"])
        acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        grid[k] = r.get("Grid_Size", "")
    mean = {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}
    count = {k: max(len(v) for v in d.values()) for k, d in acc.items()}
    return mean, count, grid


def requests(rd_path: str, wr_path: str, top: int = 40) -> None:
    rd, n, grid = _means(rd_path)
    wr, _, _ = _means(wr_path)
    print("L2->memory requests per dispatch (means) and the bytes they carry (MB = 1e6 B)")
    print(f"{'kernel':58s} {'n':>5s} {'rd128':>11s} {'rd64':>9s} {'rd32':>9s} {'read_MB':>9s} "
          f"{'wr64':>10s} {'wr32':>9s} {'write_MB':>9s} {'total_MB':>9s} {'grid':>10s}")
    rows = []
    for k, d in rd.items():
        if k not in wr:
            continue
        r128 = d.get("TCC_EA0_RDREQ_128B_sum", 0.0)
        r64 = d.get("TCC_EA0_RDREQ_64B_sum", 0.0)
        r32 = d.get("TCC_EA0_RDREQ_32B_sum", 0.0)
        w64 = wr[k].get("TCC_EA0_WRREQ_64B_sum", 0.0)
        w32 = max(wr[k].get("TCC_EA0_WRREQ_sum", 0.0) - w64, 0.0)
        rb = (128 * r128 + 64 * r64 + 32 * r32) / 1e6
        wb = (64 * w64 + 32 * w32) / 1e6
        rows.append((rb + wb, k, r128, r64, r32, rb, w64, w32, wb))
    for tot, k, r128, r64, r32, rb, w64, w32, wb in sorted(rows, key=lambda t: -t[0])[:top]:
        print(f"{k[:58]:58s} {n[k]:5d} {r128:11.0f} {r64:9.0f} {r32:9.0f} {rb:9.2f} {w64:10.0f} {w32:9.0f} "
              f"{wb:9.2f} {tot:9.2f} {grid[k]:>10s}")


def grids(path: str, top: int = 40) -> None:
    acc = collections.defaultdict(lambda: [0, 0.0])
    tot = 0.0
    for r in csv.DictReader(open(path)):
        d = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        k = (_short(r["Kernel_Name"]), r.get("Grid_Size", r.get("Grid_Size_X", "")))
        acc[k][0] += 1
        acc[k][1] += d
        tot += d
    print(f"{'kernel':50s} {'grid':>10s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>9s} {'pct':>6s}")
    for (k, g), (n, t) in sorted(acc.items(), key=lambda kv: -kv[1][1])[:top]:
        print(f"{k[:50]:50s} {g:>10s} {n:7d} {t / 1e6:10.3f} {t / n / 1e3:9.2f} {100 * t / tot:6.2f}")
    print(f"total kernel time {tot / 1e6:.3f} ms")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25)
    elif sys.argv[1] == "grids":
        grids(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 40)
    elif sys.argv[1] == "requests":
        requests(sys.argv[2], sys.argv[3], int(sys.argv[4]) if len(sys.argv) > 4 else 40)
    else:
        counter(sys.argv[2], sys.argv[3])
