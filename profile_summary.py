"""Prints a short text summary of a rocprofv3 results database: per-kernel
call counts and durations (from --kernel-trace --stats runs) and, when the
run collected them, per-dispatch PMC counter values.

usage: python3 profile_summary.py RESULTS.db [--pmc COUNTER ...]
"""
from __future__ import annotations

import argparse
import sqlite3


def kernel_table(con) -> list[tuple]:
    """(name, calls, total us, average us, percent) from the per-dispatch
    kernel records (their durations are in ns)."""
    rows = list(con.execute("select name, count(*), sum(duration), avg(duration) from kernels group by name "
                            "order by sum(duration) desc"))
    total = sum(r[2] for r in rows) or 1
    return [(n, c, t / 1e3, a / 1e3, 100.0 * t / total) for n, c, t, a in rows]


def pmc_table(con, counters) -> list[tuple]:
    rows = []
    for cname in counters:
        q = ("select kernel_name, count(*), avg(value), sum(value) from counters_collection "
             "where counter_name = ? group by kernel_name order by sum(value) desc")
        for r in con.execute(q, (cname,)):
            rows.append((cname,) + tuple(r))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--pmc", nargs="*", default=[])
    args = ap.parse_args()
    con = sqlite3.connect(args.db)
    if args.pmc:
        print("counter | kernel | dispatches | mean per dispatch | total")
        for r in pmc_table(con, args.pmc):
            print(f"{r[0]} | {r[1][:90]} | {r[2]} | {r[3]:.6g} | {r[4]:.6g}")
        return
    print("kernel | calls | total us | average us | percent")
    for name, calls, tot, avg, pct in kernel_table(con):
        print(f"{name[:100]} | {calls} | {tot:.0f} | {avg:.1f} | {pct:.2f}")


if __name__ == "__main__":
    main()
