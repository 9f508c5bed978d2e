"""Summaries of rocprofv3 CSV output for the profiles/ directory.

Two kinds of summary are written, both short text:

* kernel trace: `rocprofv3 --kernel-trace --stats --output-format csv` gives
  *_kernel_stats.csv (calls, total / average / min / max duration per kernel);
* HBM traffic of one kernel: two `rocprofv3 --pmc` runs (FETCH_SIZE, then
  WRITE_SIZE, KiB per dispatch) of the workload and two of a plain copy kernel of
  known size.  The copy runs give the factor from counter value to bytes (this GPU's
  FETCH_SIZE counts half of the bytes a streaming copy reads), which scales the
  workload's counters.

Usage (host side, after the GPU runs):
  python -m paper_2112_10223_amd.profiling trace STATS_CSV OUT.txt "COMMAND"
  python -m paper_2112_10223_amd.profiling traffic KERNEL_SUBSTR FETCH_CSV WRITE_CSV \\
      COPY_FETCH_CSV COPY_WRITE_CSV COPY_BYTES ALG_BYTES SOURCE_SHA OUT.md "COMMANDS"
  python -m paper_2112_10223_amd.profiling timeline KERNEL_TRACE_CSV OUT.txt "COMMAND"
"""
from __future__ import annotations

import csv
import sys


def _col(row: dict, *keys: str) -> str:
    low = {k.lower(): k for k in row}
    for key in keys:
        if key.lower() in low:
            return row[low[key.lower()]]
    raise KeyError(f"none of {keys} in {list(row)}")


def kernel_stats(path: str) -> list[dict]:
    out = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            out.append({
                "name": _col(row, "Name", "Kernel_Name"),
                "calls": int(_col(row, "Calls")),
                "total_ns": float(_col(row, "TotalDurationNs", "Total_Duration_Ns")),
                "avg_ns": float(_col(row, "AverageNs", "Average_Ns")),
                "min_ns": float(_col(row, "MinNs", "Min_Ns")),
                "max_ns": float(_col(row, "MaxNs", "Max_Ns")),
            })
    out.sort(key=lambda r: -r["total_ns"])
    return out


def counter_per_dispatch(path: str, kernel_substr: str) -> tuple[float, int]:
    """Mean counter value per dispatch (and dispatch count) of the kernels whose name
    contains kernel_substr; one counter per file."""
    vals = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = _col(row, "Kernel_Name", "Kernel-Name", "KernelName")
            if kernel_substr not in name:
                continue
            disp = _col(row, "Dispatch_Id", "Dispatch-Id", "DispatchId")
            vals[disp] = vals.get(disp, 0.0) + float(_col(row, "Counter_Value", "Counter-Value", "CounterValue"))
    if not vals:
        raise ValueError(f"no dispatch of a kernel matching {kernel_substr!r} in {path}")
    return sum(vals.values()) / len(vals), len(vals)


def write_trace_summary(stats_csv: str, out: str, command: str, top: int = 16) -> None:
    rows = kernel_stats(stats_csv)
    with open(out, "w") as f:
        f.write(f"# rocprofv3 kernel trace summary\n# command: {command}\n")
        f.write(f"{'kernel':<60} {'calls':>6} {'avg_us':>9} {'min_us':>9} {'max_us':>9} {'total_ms':>9}\n")
        for r in rows[:top]:
            name = r["name"].replace("void ", "")[:60]
            f.write(f"{name:<60} {r['calls']:>6} {r['avg_ns'] / 1e3:>9.2f} {r['min_ns'] / 1e3:>9.2f} "
                    f"{r['max_ns'] / 1e3:>9.2f} {r['total_ns'] / 1e6:>9.3f}\n")


def write_traffic_summary(kernel_substr: str, fetch_csv: str, write_csv: str, copy_fetch_csv: str,
                          copy_write_csv: str, copy_bytes: int, alg_bytes: int, source_sha: str, out: str,
                          commands: str) -> dict:
    fetch_kib, nf = counter_per_dispatch(fetch_csv, kernel_substr)
    write_kib, nw = counter_per_dispatch(write_csv, kernel_substr)
    # the copy kernel: the largest dispatch of an elementwise kernel (the fill runs once)
    cf, _ = _largest(copy_fetch_csv)
    cw, _ = _largest(copy_write_csv)
    f_factor = copy_bytes / (cf * 1024.0)
    w_factor = copy_bytes / (cw * 1024.0)
    traffic = fetch_kib * 1024.0 * f_factor + write_kib * 1024.0 * w_factor
    rec = {"kernel": kernel_substr, "fetch_kib_per_dispatch": round(fetch_kib, 1), "dispatches": nf,
           "write_kib_per_dispatch": round(write_kib, 1), "copy_bytes": copy_bytes,
           "copy_fetch_kib": round(cf, 1), "copy_write_kib": round(cw, 1),
           "fetch_factor": round(f_factor, 4), "write_factor": round(w_factor, 4),
           "traffic_bytes_per_launch": int(traffic), "alg_bytes_per_launch": alg_bytes,
           "traffic_over_alg": round(traffic / alg_bytes, 4) if alg_bytes else None, "source_sha": source_sha}
    with open(out, "w") as f:
        f.write(f"# HBM traffic of `{kernel_substr}` (rocprofv3 PMC)\n\ncommands:\n{commands}\n\n")
        for key, val in rec.items():
            f.write(f"{key}: {val}\n")
    return rec


def run_timeline(trace_csv: str, start_substr: str = "k_batch_init", member_prefixes=("spk::k_batch", "__amd_rocclr")):
    """Device timeline of batched runs from `--kernel-trace` output: a run starts at a
    dispatch whose name contains start_substr and takes the following dispatches whose
    names start with one of member_prefixes.  Per run: span (first start to last end),
    busy (sum of the dispatch durations) and the gaps between them."""
    rows = []
    with open(trace_csv, newline="") as f:
        for row in csv.DictReader(f):
            name = _col(row, "Kernel_Name", "Kernel-Name", "KernelName")
            rows.append((int(_col(row, "Start_Timestamp")), int(_col(row, "End_Timestamp")),
                         name[5:] if name.startswith("void ") else name))
    rows.sort()
    runs, cur = [], None
    for s, e, name in rows:
        if start_substr in name:
            if cur:
                runs.append(cur)
            cur = [(s, e, name)]
        elif cur is not None and name.startswith(member_prefixes):
            cur.append((s, e, name))
        elif cur is not None:
            runs.append(cur)
            cur = None
    if cur:
        runs.append(cur)
    out = []
    for r in runs:
        span = r[-1][1] - r[0][0]
        busy = sum(e - s for s, e, _ in r)
        out.append({"dispatches": len(r), "span_us": span / 1e3, "busy_us": busy / 1e3, "gaps_us": (span - busy) / 1e3,
                    "kernels": [(n, (e - s) / 1e3) for s, e, n in r]})
    return out


def write_timeline_summary(trace_csv: str, out: str, command: str) -> dict:
    runs = run_timeline(trace_csv)
    if not runs:
        raise ValueError(f"no batched run in {trace_csv}")
    span = sorted(r["span_us"] for r in runs)
    busy = sorted(r["busy_us"] for r in runs)
    gaps = sorted(r["gaps_us"] for r in runs)

    def pct(v, q):
        return v[min(len(v) - 1, int(round(q / 100 * (len(v) - 1))))]

    rec = {"runs": len(runs), "dispatches_per_run_median": int(pct(sorted(r["dispatches"] for r in runs), 50)),
           "span_us_p50": round(pct(span, 50), 1), "span_us_p90": round(pct(span, 90), 1),
           "busy_us_p50": round(pct(busy, 50), 1), "gaps_us_p50": round(pct(gaps, 50), 1),
           "gaps_us_p90": round(pct(gaps, 90), 1),
           "busy_share_all_runs": round(sum(busy) / max(sum(span), 1e-9), 4)}
    big = max(runs, key=lambda r: r["span_us"])
    with open(out, "w") as f:
        f.write(f"# device timeline of batched runs (rocprofv3 kernel trace)\n# command: {command}\n")
        f.write("# a run: k_batch_init and the batched-run dispatches after it; span = first start to last end,\n"
                "# busy = sum of dispatch durations, gaps = span - busy (launch gaps inside the replayed graph)\n")
        for key, val in rec.items():
            f.write(f"{key}: {val}\n")
        f.write(f"\nlongest run ({big['span_us']:.1f} us span, {big['busy_us']:.1f} us busy):\n")
        for name, us in big["kernels"]:
            f.write(f"  {name.replace('void ', '')[:70]:<70} {us:>9.1f} us\n")
    return rec


def _largest(path: str) -> tuple[float, str]:
    best, name = 0.0, ""
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            v = float(_col(row, "Counter_Value", "Counter-Value", "CounterValue"))
            if v > best:
                best, name = v, _col(row, "Kernel_Name", "Kernel-Name", "KernelName")
    return best, name


def read_traffic_summary(path: str) -> dict:
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(("#", " ", "commands")):
                key, _, val = line.partition(":")
                rec[key.strip()] = val.strip()
    return rec


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        write_trace_summary(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "timeline":
        print(write_timeline_summary(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "traffic":
        k, fc, wc, cfc, cwc, cb, ab, sha, out, cmds = sys.argv[2:12]
        print(write_traffic_summary(k, fc, wc, cfc, cwc, int(cb), int(ab), sha, out, cmds))
    else:
        raise SystemExit(__doc__)
