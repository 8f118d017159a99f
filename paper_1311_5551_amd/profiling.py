"""Reduction of rocprofv3 CSV output (kernel trace, counter collection) to per-launch figures of
one kernel over a window of its dispatches: the bench's timed region is the last N dispatches
of a kernel in the profiled bench command.

  python -m paper_1311_5551_amd.profiling trace   --csv T --kernel NAME --last N
  python -m paper_1311_5551_amd.profiling counters --csv C --kernel NAME --last N
  python -m paper_1311_5551_amd.profiling traffic --fetch F --write W --copy-fetch CF --copy-write CW \\
         --kernel NAME --last N [--out JSON --source-hash H --bench-window A..B]

HBM traffic: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the kernel, each divided by the
ratio the same counter reads for a plain device copy of known size (the runtime's copy kernel,
bytes read = bytes written = the copy size) to the copy's true bytes.
"""
from __future__ import annotations

import argparse
import csv
import json
import statistics


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def trace_window(path: str, kernel: str, last: int) -> dict:
    """Durations (ns) of the last `last` dispatches whose name contains `kernel`."""
    rows = [r for r in _rows(path) if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    win = rows[-last:] if last else rows
    d = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in win]
    return {"kernel": win[0]["Kernel_Name"] if win else kernel, "dispatches_total": len(rows), "window": len(win),
            "mean_ns": statistics.mean(d) if d else 0.0, "median_ns": statistics.median(d) if d else 0.0,
            "min_ns": min(d) if d else 0, "max_ns": max(d) if d else 0, "total_ns": sum(d)}


def counter_window(path: str, counter: str, kernel: str, last: int) -> dict:
    """Mean value per dispatch of `counter` over the last `last` dispatches of `kernel`."""
    rows = [r for r in _rows(path) if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    win = rows[-last:] if last else rows
    v = [float(r["Counter_Value"]) for r in win]
    return {"counter": counter, "window": len(win), "mean": statistics.mean(v) if v else 0.0}


def counters_window(path: str, kernel: str, last: int) -> dict:
    """Mean per dispatch of every counter in a counter-collection CSV over the last `last`
    dispatches of `kernel`."""
    rows = [r for r in _rows(path) if kernel in r["Kernel_Name"]]
    ids = sorted(set(int(r["Dispatch_Id"]) for r in rows))
    keep = set(ids[-last:] if last else ids)
    out = {"kernel": rows[0]["Kernel_Name"] if rows else kernel, "dispatches_total": len(ids), "window": len(keep)}
    acc = {}
    for r in rows:
        if int(r["Dispatch_Id"]) in keep:
            acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    for k, v in sorted(acc.items()):
        out[k] = sum(v) / len(keep)
    return out


def copy_factor(path: str, counter: str, bytes_per_copy: int, kernel: str = "copyBuffer") -> float:
    """Counter reading (KiB) per true byte of a plain copy: mean over the copy dispatches / size."""
    c = counter_window(path, counter, kernel, 0)
    return c["mean"] * 1024.0 / bytes_per_copy


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--csv", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--last", type=int, default=0)
    q = sub.add_parser("counters")
    q.add_argument("--csv", required=True)
    q.add_argument("--kernel", required=True)
    q.add_argument("--last", type=int, default=0)
    c = sub.add_parser("traffic")
    for k in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--kernel"):
        c.add_argument(k, required=True)
    c.add_argument("--last", type=int, default=0)
    c.add_argument("--copy-bytes", type=int, default=1 << 30)
    c.add_argument("--out")
    c.add_argument("--source-hash")
    c.add_argument("--bench-window", help="the bench's timed steps, e.g. 9990..10010")
    c.add_argument("--copy-kernel", default="copyBuffer", help="name of the plain copy kernel in the copy runs")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(json.dumps(trace_window(a.csv, a.kernel, a.last), indent=1))
        return
    if a.cmd == "counters":
        print(json.dumps(counters_window(a.csv, a.kernel, a.last), indent=1))
        return
    ff = copy_factor(a.copy_fetch, "FETCH_SIZE", a.copy_bytes, a.copy_kernel)
    fw = copy_factor(a.copy_write, "WRITE_SIZE", a.copy_bytes, a.copy_kernel)
    fe = counter_window(a.fetch, "FETCH_SIZE", a.kernel, a.last)
    wr = counter_window(a.write, "WRITE_SIZE", a.kernel, a.last)
    res = {"kernel": a.kernel, "window": fe["window"], "fetch_kib_per_launch": fe["mean"],
           "write_kib_per_launch": wr["mean"], "copy_fetch_counted_per_byte": ff,
           "copy_write_counted_per_byte": fw,
           "bytes_read_per_launch": fe["mean"] * 1024.0 / ff, "bytes_written_per_launch": wr["mean"] * 1024.0 / fw}
    res["bytes_per_launch"] = res["bytes_read_per_launch"] + res["bytes_written_per_launch"]
    if a.source_hash:
        res["source_hash"] = a.source_hash
    if a.bench_window:
        res["bench_window"] = a.bench_window
    print(json.dumps(res, indent=1))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
