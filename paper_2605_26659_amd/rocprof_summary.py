"""Summaries of rocprofv3 output databases (rocpd SQLite files).

    python -m paper_2605_26659_amd.rocprof_summary DB [DB ...] [--top N]

For each database: per kernel, the dispatch count, mean / min / max duration
(kernel trace) and the per-dispatch mean of every collected counter (PMC
runs). Prints plain text suitable for committing as a profile summary.
"""
from __future__ import annotations

import argparse
import collections
import sqlite3


def kernel_stats(db: str, top: int = 15):
    con = sqlite3.connect(db)
    cur = con.cursor()
    out = []
    try:
        rows = cur.execute(
            "select name, count(*), avg(end-start), min(end-start), max(end-start), sum(end-start) "
            "from kernels group by name order by sum(end-start) desc").fetchall()
    except sqlite3.Error:
        rows = []
    for name, n, avg, mn, mx, tot in rows[:top]:
        out.append((name, n, avg / 1e3, mn / 1e3, mx / 1e3, tot / 1e6))
    return out


def counter_stats(db: str):
    con = sqlite3.connect(db)
    cur = con.cursor()
    try:
        rows = cur.execute("select kernel_name, counter_name, avg(value), count(*) "
                           "from counters_collection group by kernel_name, counter_name").fetchall()
    except sqlite3.Error:
        return {}
    by = collections.defaultdict(dict)
    for k, c, v, n in rows:
        by[k][c] = (v, n)
    return by


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("dbs", nargs="+")
    ap.add_argument("--top", type=int, default=15)
    a = ap.parse_args(argv)
    for db in a.dbs:
        print(f"== {db}")
        ks = kernel_stats(db, a.top)
        if ks:
            print(f"{'dispatches':>10} {'avg_us':>10} {'min_us':>9} {'max_us':>9} {'total_ms':>10}  kernel")
            for name, n, avg, mn, mx, tot in ks:
                print(f"{n:>10d} {avg:>10.2f} {mn:>9.2f} {mx:>9.2f} {tot:>10.2f}  {name[:120]}")
        cs = counter_stats(db)
        for k, d in sorted(cs.items(), key=lambda kv: -max(n for _, n in kv[1].values())):
            n = max(c for _, c in d.values())
            print(f"{n:>10d}  {k[:120]}")
            for c, (v, _) in sorted(d.items()):
                print(f"{'':>12}{c:<24} {v:.6g}")


if __name__ == "__main__":
    main()
