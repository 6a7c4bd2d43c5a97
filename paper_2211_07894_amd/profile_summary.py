"""Short summaries of rocprofv3 output.

    python -m paper_2211_07894_amd.profile_summary trace RESULTS.db "COMMAND" [--top 15] \
        [--shapes REGEX]
        Markdown table of kernels by total GPU time from a --kernel-trace run
        (rocpd SQLite, ROCm 7): calls, total and average duration, share; with
        --shapes, also per launch shape (grid size) of the matching kernels.

    python -m paper_2211_07894_amd.profile_summary traffic --fetch F.csv --write W.csv \
        --form bf16x3 --workload c64_n1024_slab --out profiles/traffic.json --command "..."
        HBM bytes per dispatch of the hot-path kernels from two --pmc runs
        (FETCH_SIZE, then WRITE_SIZE, both in KiB per dispatch), each scaled by
        what the same counter reads for the calibration copy (bench.py
        --copy-calibration: three elementwise passes reading and writing 1 GiB).

    python -m paper_2211_07894_amd.profile_summary sq COUNTERS.csv "COMMAND" \
        [--kernels REGEX] [--title TEXT]
        Markdown table of SQ counters per dispatch (mean over the run's dispatches
        of each kernel), with VALU instructions per MFMA instruction and the MFMA
        busy share of SQ_BUSY_CYCLES where those counters were collected.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sqlite3
import statistics
import sys

PKG = os.path.dirname(os.path.abspath(__file__))

# profiling-scope name -> (kernel-name pattern, source file) for each storage form
KERNELS = {
    "fp64": {"proj": (r"tn_sym_f64_kernel<double, double>", "gemm.hip"),
             "backproj": (r"backproj_f64_kernel", "gemm.hip"),
             "cheb_step": (r"cheb_vec_kernel<double|cheb_plane_kernel<double, double", "stencil.hip"),
             "cheb_pair": (r"cheb_pair_kernel<double", "stencil.hip"),
             "cheb_triple": (r"cheb_multi_kernel<double", "stencil.hip")},
    "fp32": {"proj": (r"tn_sym_pipe_kernel<.*true>", "gemm_lp.hip"),
             "backproj": (r"backproj_pipe_kernel", "gemm_lp.hip"),
             "cheb_step": (r"cheb_vec_kernel<float|cheb_plane_kernel<float, float", "stencil.hip"),
             "cheb_pair": (r"cheb_pair_kernel<float", "stencil.hip"),
             "cheb_triple": (r"cheb_multi_kernel<float", "stencil.hip")},
    "bf16x3": {"proj": (r"tn_sym_p3_kernel|tn_sym_pipe_kernel<.*true>", "gemm_lp.hip"),
               "backproj": (r"backproj_p3w_kernel|backproj_p3_kernel|backproj_pipe_kernel", "gemm_lp.hip"),
               "cheb_step": (r"cheb_vec_kernel<float|cheb_plane_kernel<float, float", "stencil.hip"),
               "cheb_pair": (r"cheb_pair_kernel<float", "stencil.hip"),
             "cheb_triple": (r"cheb_multi_kernel<float", "stencil.hip")},
}
CALIBRATION_BYTES = 1 << 30


def short(name: str) -> str:
    """Kernel name without namespace noise and without its argument list (the
    last balanced parenthesised group; template arguments may hold parentheses)."""
    name = name.replace("lrdm::(anonymous namespace)::", "").replace("void ", "").strip()
    if name.endswith(")"):
        depth = 0
        for i in range(len(name) - 1, -1, -1):
            depth += {")": 1, "(": -1}.get(name[i], 0)
            if depth == 0:
                return name[:i]
    return name


def trace_summary(db_path: str, command: str, top: int = 15, shapes: str = "") -> str:
    db = sqlite3.connect(db_path)
    rows = list(db.execute(
        "select name, total_calls, total_duration, average, percentage from top_kernels"))
    total_us = sum(r[2] for r in rows)          # the top_kernels view reports microseconds
    out = [f"Command: `{command}`", "",
           f"Total kernel time: {total_us / 1e3:.1f} ms over {sum(r[1] for r in rows)} dispatches",
           "", "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, calls, tot, avg, pct in rows[:top]:
        out.append(f"| {short(name)} | {calls} | {tot / 1e3:.2f} | {avg:.1f} | {pct:.2f} |")
    if shapes:
        # one kernel runs in several launch shapes (the bench's 16-direction call,
        # single directions of the low-rank step, the tuner's trial split counts):
        # per shape, so that a launch can be matched to the bench's live figure
        out += ["", "Launch shapes of the kernels matching `" + shapes + "` (grid in threads, "
                "durations in nanoseconds as recorded):", "",
                "| kernel | grid | workgroup | calls | avg ms | min ms | max ms |",
                "|---|---:|---:|---:|---:|---:|---:|"]
        q = ("select name, grid_x, workgroup_x, count(*), avg(duration), min(duration), "
             "max(duration) from kernels group by name, grid_x, workgroup_x "
             "order by name, grid_x")
        for name, gx, wx, n, avg, lo, hi in db.execute(q):
            if re.search(shapes, short(name)):
                out.append(f"| {short(name)} | {gx} | {wx} | {n} | {avg / 1e6:.3f} | "
                           f"{lo / 1e6:.3f} | {hi / 1e6:.3f} |")
    return "\n".join(out) + "\n"


def _col(header, *keys):
    for k in keys:
        for i, h in enumerate(header):
            if h.strip().lower() == k.lower():
                return i
    raise KeyError(f"none of {keys} in {header}")


def read_counter(path: str, counter: str):
    """{dispatch id: (kernel name, value summed over the rows of that dispatch)}."""
    with open(path, newline="") as f:
        rd = csv.reader(f)
        header = next(rd)
        i_d = _col(header, "Dispatch_Id", "Dispatch_ID")
        i_k = _col(header, "Kernel_Name")
        i_c = _col(header, "Counter_Name")
        i_v = _col(header, "Counter_Value")
        out = {}
        for row in rd:
            if row[i_c] != counter:
                continue
            d = int(row[i_d])
            name, v = out.get(d, (row[i_k], 0.0))
            out[d] = (name, v + float(row[i_v]))
    return out


def _source_sha(name: str) -> str:
    p = os.path.join(PKG, "csrc", name)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic(fetch_csv, write_csv, form, workload, command):
    recs = []
    data = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        disp = read_counter(path, counter)
        cal = sorted((v for n, v in disp.values() if "elementwise" in n), reverse=True)[:3]
        if not cal:
            raise SystemExit(f"no calibration copy dispatches in {path}")
        kib = statistics.median(cal)
        factor = CALIBRATION_BYTES / (kib * 1024.0)   # true bytes per counted byte
        data[counter] = (disp, factor, kib)
    table = KERNELS[form]
    for scope, (pat, src) in table.items():
        per = {}
        for counter, (disp, factor, _) in data.items():
            vals = [v for n, v in disp.values() if re.search(pat, short(n))]
            if vals:
                per[counter] = statistics.median(vals) * 1024.0 * factor
        if len(per) == 2:
            recs.append({
                "kernel": scope, "workload": workload, "form": form, "source": src,
                "source_sha": _source_sha(src),
                "fetch_bytes_per_launch": round(per["FETCH_SIZE"]),
                "write_bytes_per_launch": round(per["WRITE_SIZE"]),
                "bytes_per_launch": round(per["FETCH_SIZE"] + per["WRITE_SIZE"]),
                "calibration": {c: {"copy_kib_counted": round(data[c][2]),
                                    "factor": round(data[c][1], 4)} for c in data},
                "command": command,
            })
    return recs


def read_counters(path: str):
    """{dispatch id: (kernel name, {counter: value summed over that dispatch's rows})}."""
    with open(path, newline="") as f:
        rd = csv.reader(f)
        header = next(rd)
        i_d = _col(header, "Dispatch_Id", "Dispatch_ID")
        i_k = _col(header, "Kernel_Name")
        i_c = _col(header, "Counter_Name")
        i_v = _col(header, "Counter_Value")
        out = {}
        for row in rd:
            d = int(row[i_d])
            name, vals = out.setdefault(d, (row[i_k], {}))
            vals[row[i_c]] = vals.get(row[i_c], 0.0) + float(row[i_v])
    return out


def sq_summary(path: str, command: str, kernels: str, title: str) -> str:
    disp = read_counters(path)
    groups = {}
    for name, vals in disp.values():
        k = short(name)
        if kernels and not re.search(kernels, k):
            continue
        groups.setdefault(k, []).append(vals)
    counters = sorted({c for vs in groups.values() for v in vs for c in v})
    head = ["kernel", "dispatches"] + counters
    derived = []
    if "SQ_INSTS_VALU" in counters and "SQ_INSTS_MFMA" in counters:
        derived.append("VALU / MFMA")
    if "SQ_VALU_MFMA_BUSY_CYCLES" in counters and "SQ_BUSY_CYCLES" in counters:
        derived.append("MFMA busy share")
    out = [f"# {title}" if title else "# SQ counters", "", f"Command: `{command}`", "",
           "Values per dispatch (mean over the dispatches of the run), as the counters "
           "report them.  MFMA busy share = (SQ_VALU_MFMA_BUSY_CYCLES / 1024 SIMDs) / "
           "(SQ_BUSY_CYCLES / 32 shader engines): the share of the kernel's cycles in "
           "which a SIMD's matrix core is busy (for kernels that occupy every shader "
           "engine).", "",
           "| " + " | ".join(head + derived) + " |",
           "|---|" + "---:|" * (len(head) - 1 + len(derived))]
    for k in sorted(groups, key=lambda k: -max(v.get("SQ_BUSY_CYCLES", 0.0) for v in groups[k])):
        vs = groups[k]
        mean = {c: statistics.mean(v.get(c, 0.0) for v in vs) for c in counters}
        row = [k, str(len(vs))] + [f"{mean[c]:.4g}" for c in counters]
        if "VALU / MFMA" in derived:
            row.append(f"{mean['SQ_INSTS_VALU'] / mean['SQ_INSTS_MFMA']:.2f}"
                       if mean["SQ_INSTS_MFMA"] else "-")
        if "MFMA busy share" in derived:
            row.append(f"{(mean['SQ_VALU_MFMA_BUSY_CYCLES'] / 1024) / (mean['SQ_BUSY_CYCLES'] / 32):.3f}"
                       if mean["SQ_BUSY_CYCLES"] else "-")
        out.append("| " + " | ".join(row) + " |")
    return "\n".join(out) + "\n"


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("command")
    t.add_argument("--top", type=int, default=15)
    t.add_argument("--shapes", default="")
    q = sub.add_parser("traffic")
    q.add_argument("--fetch", required=True)
    q.add_argument("--write", required=True)
    q.add_argument("--form", required=True)
    q.add_argument("--workload", required=True)
    q.add_argument("--out", required=True)
    q.add_argument("--command", required=True)
    c = sub.add_parser("sq")
    c.add_argument("csv")
    c.add_argument("command")
    c.add_argument("--kernels", default="")
    c.add_argument("--title", default="")
    a = ap.parse_args(argv)
    if a.mode == "sq":
        sys.stdout.write(sq_summary(a.csv, a.command, a.kernels, a.title))
        return 0
    if a.mode == "trace":
        sys.stdout.write(trace_summary(a.db, a.command, a.top, a.shapes))
        return 0
    recs = traffic(a.fetch, a.write, a.form, a.workload, a.command)
    old = []
    if os.path.exists(a.out):
        old = [r for r in json.load(open(a.out))
               if not (r.get("form") == a.form and r.get("workload") == a.workload)]
    json.dump(old + recs, open(a.out, "w"), indent=1)
    for r in recs:
        print(f"{r['kernel']}: fetch {r['fetch_bytes_per_launch'] / 1e9:.3f} GB, "
              f"write {r['write_bytes_per_launch'] / 1e9:.3f} GB per launch")
    return 0


if __name__ == "__main__":
    sys.exit(main())
