"""Turn a rocprofv3 database (rocpd SQLite, ROCm 7) into a short Markdown
kernel summary.

    python -m paper_2211_07894_amd.profile_summary RESULTS.db "COMMAND" [--top 15]

Prints a table of kernels by total GPU time: calls, total and average
duration, share of the total.
"""
from __future__ import annotations

import argparse
import re
import sqlite3
import sys


def short(name: str) -> str:
    name = name.replace("lrdm::(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", name)


def summary(db_path: str, command: str, top: int = 15) -> str:
    db = sqlite3.connect(db_path)
    rows = list(db.execute(
        "select name, total_calls, total_duration, average, percentage from top_kernels"))
    total_us = sum(r[2] for r in rows)          # the top_kernels view reports microseconds
    out = [f"Command: `{command}`", "",
           f"Total kernel time: {total_us / 1e3:.1f} ms over {sum(r[1] for r in rows)} dispatches",
           "", "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, calls, tot, avg, pct in rows[:top]:
        out.append(f"| {short(name)} | {calls} | {tot / 1e3:.2f} | {avg:.1f} | {pct:.2f} |")
    return "\n".join(out) + "\n"


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("command")
    ap.add_argument("--top", type=int, default=15)
    a = ap.parse_args(argv)
    sys.stdout.write(summary(a.db, a.command, a.top))
    return 0


if __name__ == "__main__":
    sys.exit(main())
