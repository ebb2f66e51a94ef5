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


def occupancy(db):
    """Span of the trace, time with at least one kernel running (union of the dispatch
    intervals) and kernel time per stream, in ns."""
    con = sqlite3.connect(db)
    rows = con.execute("select start, end, stream from kernels order by start").fetchall()
    if not rows:
        return 0, 0, {}
    busy, cur_s, cur_e = 0, rows[0][0], rows[0][1]
    per_stream = {}
    for s, e, st in rows:
        per_stream[st] = per_stream.get(st, 0) + (e - s)
        if s > cur_e:
            busy += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    busy += cur_e - cur_s
    span = max(e for _, e, _ in rows) - rows[0][0]
    return span, busy, per_stream


def counters(db):
    """{(kernel, counter): [dispatches, mean value per dispatch, mean duration ns]}."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, counter_name, counter_value, duration from pmc_events").fetchall()
    agg = {}
    for n, c, v, d in rows:
        a = agg.setdefault((short_name(n), c), [0, 0.0, 0.0])
        a[0] += 1
        a[1] += v
        a[2] += d
    return {k: [c, s / c, d / c] for k, (c, s, d) in agg.items()}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=20)
    ap.add_argument("--busy", action="store_true", help="also print span, busy time, streams")
    ap.add_argument("--pmc", action="store_true", help="print counter values per dispatch")
    a = ap.parse_args(argv)
    if a.pmc:
        print(f"{'kernel':52s} {'counter':12s} {'dispatches':>10s} {'mean/dispatch':>16s} {'mean us':>10s}")
        for (n, c), (cnt, v, d) in sorted(counters(a.db).items()):
            print(f"{n[:52]:52s} {c:12s} {cnt:10d} {v:16.1f} {d / 1e3:10.1f}")
        return
    if a.busy:
        span, busy, per_stream = occupancy(a.db)
        print(f"trace span {span / 1e6:.1f} ms, device busy (any kernel running) "
              f"{busy / 1e6:.1f} ms = {100 * busy / max(span, 1):.1f} %")
        for st, t in sorted(per_stream.items(), key=lambda x: -x[1]):
            print(f"  stream {st}: kernel time {t / 1e6:.1f} ms")
    agg = summarize(a.db)
    tot = sum(v[1] for v in agg.values())
    print(f"{'kernel':64s} {'calls':>7s} {'total ms':>10s} {'avg us':>10s} {'%':>6s}")
    for n, (c, t) in sorted(agg.items(), key=lambda x: -x[1][1])[: a.top]:
        print(f"{n[:64]:64s} {c:7d} {t / 1e6:10.2f} {t / c / 1e3:10.2f} {100 * t / tot:6.1f}")
    print(f"total kernel time {tot / 1e6:.2f} ms")


if __name__ == "__main__":
    main()
