"""Summaries of rocprofv3 output for the stereomesh kernels.

``python -m paper_1511_00758_amd.profiling stats <kernel_stats.csv> --cmd "<command>"``
prints a Markdown table of a ``--kernel-trace --stats`` run;
``python -m paper_1511_00758_amd.profiling traffic ...`` turns two ``--pmc`` runs
(FETCH_SIZE, WRITE_SIZE, in KiB per dispatch) of a kernel, plus the same two
counters read on a plain copy of known size, into HBM bytes per launch.
"""
import argparse
import csv
import json
import os
import sys


def short_name(name: str) -> str:
    n = name.replace("sm::(anonymous namespace)::", "").replace("void ", "")
    return n.split("(")[0].strip()


def kernel_stats_rows(path):
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            rows.append({"name": short_name(r["Name"]), "calls": int(r["Calls"]),
                         "avg_us": float(r["AverageNs"]) / 1e3, "min_us": float(r["MinNs"]) / 1e3,
                         "max_us": float(r["MaxNs"]) / 1e3, "total_us": float(r["TotalDurationNs"]) / 1e3,
                         "pct": float(r["Percentage"])})
    return rows


def trace_stats_rows(path, skip_solves):
    """Per-kernel statistics of a ``--kernel-trace`` CSV over the dispatches after the
    ``skip_solves``-th end-of-solve read-back (one ``copyBuffer`` per solve): the frames of
    a run, without the solves of the autotuner before them."""
    recs = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            recs.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    recs.sort()
    seen, start = 0, 0
    for i, (_, _, name) in enumerate(recs):
        if seen == skip_solves:
            start = i
            break
        if "copyBuffer" in name:
            seen += 1
    per = {}
    for t0, t1, name in recs[start:]:
        per.setdefault(short_name(name), []).append((t1 - t0) / 1e3)
    total = sum(sum(v) for v in per.values()) or 1.0
    rows = [{"name": k, "calls": len(v), "avg_us": sum(v) / len(v), "min_us": min(v), "max_us": max(v),
             "total_us": sum(v), "pct": 100.0 * sum(v) / total} for k, v in per.items()]
    return sorted(rows, key=lambda r: -r["total_us"])


def kernel_stats_md(path, cmd, title, rows=None, note=None):
    rows = kernel_stats_rows(path) if rows is None else rows
    out = [f"# {title}", "", "Command:", "", "```", cmd, "```", ""]
    if note:
        out += [note, ""]
    out += ["| kernel | calls | avg us | min us | max us | total us | % |",
            "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| {r['name']} | {r['calls']} | {r['avg_us']:.2f} | {r['min_us']:.2f} | "
                   f"{r['max_us']:.2f} | {r['total_us']:.0f} | {r['pct']:.1f} |")
    return "\n".join(out) + "\n"


def counter_per_dispatch(path, kernel_substr, counter):
    """Mean value of ``counter`` over the dispatches whose kernel name contains
    ``kernel_substr`` (rocprofv3 counter_collection.csv)."""
    vals = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if counter not in r.get("Counter_Name", ""):
                continue
            if kernel_substr in r.get("Kernel_Name", ""):
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise ValueError(f"no {counter} rows for {kernel_substr} in {path}")
    return sum(vals) / len(vals), len(vals)


def traffic(fetch_csv, write_csv, kernel, calib_fetch_csv, calib_write_csv, calib_kernel, calib_bytes):
    f_kib, nf = counter_per_dispatch(fetch_csv, kernel, "FETCH_SIZE")
    w_kib, nw = counter_per_dispatch(write_csv, kernel, "WRITE_SIZE")
    cf_kib, _ = counter_per_dispatch(calib_fetch_csv, calib_kernel, "FETCH_SIZE")
    cw_kib, _ = counter_per_dispatch(calib_write_csv, calib_kernel, "WRITE_SIZE")
    kf = calib_bytes / (cf_kib * 1024.0)
    kw = calib_bytes / (cw_kib * 1024.0)
    return {"kernel": kernel, "fetch_kib_raw": f_kib, "write_kib_raw": w_kib, "dispatches": [nf, nw],
            "copy_calibration": {"bytes": calib_bytes, "fetch_kib": cf_kib, "write_kib": cw_kib,
                                 "fetch_factor": kf, "write_factor": kw},
            "bytes_per_launch": f_kib * 1024.0 * kf + w_kib * 1024.0 * kw}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="action", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", default="rocprofv3 kernel statistics")
    s.add_argument("--trace", default=None, help="kernel_trace.csv: statistics from the trace instead")
    s.add_argument("--skip-solves", type=int, default=0,
                   help="with --trace: only the dispatches after this many solves (the autotuner's)")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--calib-fetch", required=True)
    t.add_argument("--calib-write", required=True)
    t.add_argument("--calib-kernel", default="copy")
    t.add_argument("--calib-bytes", type=float, required=True)
    t.add_argument("--source-hash", default=None)
    t.add_argument("--cmd", default="")
    a = ap.parse_args(argv)
    if a.action == "stats":
        if a.trace:
            note = (f"From the kernel trace, after the first {a.skip_solves} solves (the autotuner's, "
                    "on the run's first frame): the frames of the run.")
            sys.stdout.write(kernel_stats_md(a.csv, a.cmd, a.title, trace_stats_rows(a.trace, a.skip_solves), note))
        else:
            sys.stdout.write(kernel_stats_md(a.csv, a.cmd, a.title))
    else:
        res = traffic(a.fetch, a.write, a.kernel, a.calib_fetch, a.calib_write, a.calib_kernel,
                      a.calib_bytes)
        res["kernel_source_hash"] = a.source_hash
        res["commands"] = a.cmd
        print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
