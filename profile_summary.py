"""Summarise a rocprofv3 results database (per-kernel calls, mean/min duration
and resources) as a markdown table."""
import sqlite3
import sys


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


if __name__ == "__main__":
    print(summarise(sys.argv[1]))
