"""Per-kernel summary of a rocprofv3 kernel trace (the SQLite results database).

    python3 -m paper_2104_01439_amd.profile_summary RUN_results.db [--top 20]

Prints, per kernel (template arguments kept, argument lists dropped): dispatches, total and
average device time and share of the total, in the same form as rocprofv3 --stats.
"""

import argparse
import re
import sqlite3


def short_name(n):
    n = n.replace("(anonymous namespace)::", "")
    m = re.match(r"(?:void )?([\w:]+)(<[^()]*>)?", n)
    return (m.group(1) + (m.group(2) or "")) if m else n


def summarize(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels").fetchall()
    agg = {}
    for n, d in rows:
        a = agg.setdefault(short_name(n), [0, 0.0])
        a[0] += 1
        a[1] += d
    return agg


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=20)
    a = ap.parse_args(argv)
    agg = summarize(a.db)
    tot = sum(v[1] for v in agg.values())
    print(f"{'kernel':64s} {'calls':>7s} {'total ms':>10s} {'avg us':>10s} {'%':>6s}")
    for n, (c, t) in sorted(agg.items(), key=lambda x: -x[1][1])[: a.top]:
        print(f"{n[:64]:64s} {c:7d} {t / 1e6:10.2f} {t / c / 1e3:10.2f} {100 * t / tot:6.1f}")
    print(f"total kernel time {tot / 1e6:.2f} ms")


if __name__ == "__main__":
    main()
