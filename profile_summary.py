"""Summarise a rocprofv3 results database: per-kernel calls, mean/min/max
duration and resources as a markdown table, and, with --iteration KEY, the
launch sequence of one iteration (the sequence that most often runs from one
dispatch of a kernel whose name contains KEY to the next) with each launch's
mean start offset and duration.

    python profile_summary.py DB [--top N] [--iteration KEY]
"""
import argparse
import sqlite3


def summarise(db: str, top: int = 25) -> str:
    con = sqlite3.connect(db)
    rows = con.execute(
        "select name, count(*), avg(duration), min(duration), max(duration), sum(duration), grid_x, workgroup_x, "
        "vgpr_count, sgpr_count, lds_size from kernels group by name order by sum(duration) desc limit ?",
        (top,),
    ).fetchall()
    total = sum(r[5] for r in rows) or 1.0
    out = ["| kernel | calls | mean us | min us | max us | share | grid | wg | vgpr | sgpr | lds B |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    for name, n, avg, mn, mx, sm, gx, wg, vg, sg, lds in rows:
        short = name.split("(")[0].replace("void ", "")
        out.append(f"| `{short}` | {n} | {avg/1e3:.2f} | {mn/1e3:.2f} | {mx/1e3:.2f} | {100*sm/total:.1f}% | "
                   f"{gx // max(wg, 1)} | {wg} | {vg} | {sg} | {lds} |")
    return "\n".join(out)


def iteration(db: str, key: str) -> str:
    """One iteration's launches: the launch sequence that most often runs from
    one dispatch of a kernel whose name contains key to the next, with each
    launch's mean start offset and duration over those occurrences."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    idx = [i for i, r in enumerate(rows) if key in r[0]]
    seqs = {}
    for a, b in zip(idx, idx[1:]):
        names = tuple(r[0] for r in rows[a:b])
        seqs.setdefault(names, []).append(a)
    if not seqs:
        return f"(fewer than two dispatches of {key})"
    names, starts = max(seqs.items(), key=lambda kv: len(kv[1]))
    k = len(names)
    span = sum(rows[a + k][1] - rows[a][1] for a in starts) / len(starts)
    out = [f"{k} launches, {span / 1e3:.1f} us start to start (mean of {len(starts)} iterations)", "",
           "| start us | duration us | kernel |", "|---|---|---|"]
    for i, name in enumerate(names):
        st = sum(rows[a + i][1] - rows[a][1] for a in starts) / len(starts)
        du = sum(rows[a + i][2] - rows[a + i][1] for a in starts) / len(starts)
        out.append(f"| {st / 1e3:.1f} | {du / 1e3:.1f} | `{name.split('(')[0].replace('void ', '')}` |")
    return "\n".join(out)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--iteration", default=None)
    a = ap.parse_args()
    print(iteration(a.db, a.iteration) if a.iteration else summarise(a.db, a.top))
