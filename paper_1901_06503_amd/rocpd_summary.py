"""Summaries of rocprofv3 result databases (rocpd SQLite) for the profile notes.

  python -m paper_1901_06503_amd.rocpd_summary kernels DB [--top N]
      per-kernel calls, total and average duration (the --stats table)
  python -m paper_1901_06503_amd.rocpd_summary pmc DB --kernel SUBSTRING
      average per-dispatch value of each collected counter for matching kernels
"""
from __future__ import annotations

import argparse
import re
import sqlite3
import statistics


def kernel_table(db_path: str, top: int = 15):
    cur = sqlite3.connect(db_path).cursor()
    rows = cur.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    out = []
    for name, calls, total, avg, pct in rows[:top]:
        out.append((re.sub(r"\(.*", "", name), int(calls), float(total) / 1e3, float(avg), float(pct)))
    return out


def pmc_means(db_path: str, kernel_substring: str):
    cur = sqlite3.connect(db_path).cursor()
    rows = cur.execute("select kernel_name, counter_name, value, dispatch_id from counters_collection").fetchall()
    per = {}
    for kname, counter, value, disp in rows:
        if kernel_substring in kname:
            per.setdefault(counter, {}).setdefault(disp, 0.0)
            per[counter][disp] += float(value)
    return {c: (len(v), statistics.mean(v.values())) for c, v in per.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["kernels", "pmc"])
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=15)
    ap.add_argument("--kernel", default="")
    a = ap.parse_args()
    if a.what == "kernels":
        print(f"{'kernel':70s} {'calls':>7s} {'total ms':>10s} {'avg us':>10s} {'%':>6s}")
        for name, calls, total, avg, pct in kernel_table(a.db, a.top):
            print(f"{name[:70]:70s} {calls:7d} {total:10.2f} {avg:10.2f} {pct:6.1f}")
    else:
        for counter, (n, mean) in sorted(pmc_means(a.db, a.kernel).items()):
            print(f"{counter}: {mean:.1f} (mean over {n} dispatches of kernels matching '{a.kernel}')")


if __name__ == "__main__":
    main()
