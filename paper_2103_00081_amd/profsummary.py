"""Summarise a rocprofv3 kernel trace (SQLite results database) per kernel.

Usage: python -m paper_2103_00081_amd.profsummary <run_results.db> [top]
Prints total device time, launch count, average / minimum duration, grid
size, VGPR count and scratch bytes for each kernel, heaviest first.
"""
import re
import sqlite3
import sys


def summarise(db: str, top: int = 40) -> str:
    c = sqlite3.connect(db)
    rows = c.execute("select name, start, end, grid_x, vgpr_count, scratch_size from kernels").fetchall()
    agg = {}
    for name, s, e, gx, vg, scr in rows:
        short = name.replace("(anonymous namespace)::", "").split("(")[0]
        short = re.sub(r"\s+", " ", short)
        a = agg.setdefault(short, [0, 0.0, 1e99, gx, vg, scr])
        a[0] += 1
        a[1] += e - s
        a[2] = min(a[2], e - s)
    tot = sum(v[1] for v in agg.values())
    out = ["total kernel time %.3f ms, %d launches" % (tot / 1e6, sum(v[0] for v in agg.values())),
           "| kernel | launches | total ms | share | avg us | min us | grid | vgpr | scratch |",
           "|---|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append("| %s | %d | %.3f | %.1f%% | %.2f | %.2f | %d | %d | %d |" % (
            k, v[0], v[1] / 1e6, 100 * v[1] / tot, v[1] / v[0] / 1e3, v[2] / 1e3, v[3], v[4], v[5]))
    return "\n".join(out)


if __name__ == "__main__":
    print(summarise(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 40))
