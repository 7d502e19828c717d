"""Summarise rocprofv3 output per kernel.

Usage:
  python -m paper_2103_00081_amd.profsummary trace <run_results.db> [top]
      total device time, launches, average / minimum duration, grid size,
      VGPR count and scratch bytes per kernel (heaviest first), then the
      fine-level operator kernels grouped by (field, precision).
  python -m paper_2103_00081_amd.profsummary pmc <counter_collection.csv | results.db> [copy_mib]
      per-dispatch hardware counters (e.g. FETCH_SIZE, WRITE_SIZE) averaged
      per operator class, epilogue and grid size; with copy_mib, the counters
      of the largest plain copy in the run (the library's stream copy of
      copy_mib MiB, read and written) give the factor from counter units to
      bytes.
"""
import csv
import re
import sqlite3
import sys

_APPLY = re.compile(r"k_q([12])_apply<(float|double), (\d)")


def short_name(name: str) -> str:
    s = name.replace("(anonymous namespace)::", "").split("(")[0]
    return re.sub(r"\s+", " ", s)


def apply_class(name: str):
    m = _APPLY.search(name)
    if not m:
        return None
    field = "pressure" if m.group(3) == "0" else "heat"
    prec = "FP64" if m.group(2) == "double" else "FP32"
    return "Q%s %s apply %s" % (m.group(1), field, prec)


def summarise(db: str, top: int = 40) -> str:
    c = sqlite3.connect(db)
    rows = c.execute("select name, start, end, grid_x, vgpr_count, scratch_size from kernels").fetchall()
    agg, cls = {}, {}
    for name, s, e, gx, vg, scr in rows:
        short = short_name(name)
        a = agg.setdefault(short, [0, 0.0, 1e99, gx, vg, scr])
        a[0] += 1
        a[1] += e - s
        a[2] = min(a[2], e - s)
        k = apply_class(name)
        if k:
            b = cls.setdefault(k, [0, 0.0])
            b[0] += 1
            b[1] += e - s
    tot = sum(v[1] for v in agg.values())
    out = ["total kernel time %.3f ms, %d launches" % (tot / 1e6, sum(v[0] for v in agg.values())), "",
           "| kernel | launches | total ms | share | avg us | min us | grid | vgpr | scratch |",
           "|---|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append("| %s | %d | %.3f | %.1f%% | %.2f | %.2f | %d | %d | %d |" % (
            k, v[0], v[1] / 1e6, 100 * v[1] / tot, v[1] / v[0] / 1e3, v[2] / 1e3, v[3], v[4], v[5]))
    out += ["", "fine-level operator kernels by class (all epilogues):", "",
            "| class | launches | total ms | share | avg us |", "|---|---|---|---|---|"]
    for k, v in sorted(cls.items(), key=lambda kv: -kv[1][1]):
        out.append("| %s | %d | %.3f | %.1f%% | %.2f |" % (k, v[0], v[1] / 1e6, 100 * v[1] / tot,
                                                         v[1] / v[0] / 1e3))
    return "\n".join(out)


def _pmc_rows(path: str):
    """(dispatch id, kernel name, grid size, counter, value) from a rocprofv3
    counter CSV or results database."""
    if path.endswith(".db"):
        c = sqlite3.connect(path)
        return c.execute("select dispatch_id, kernel_name, grid_size, counter_name, value "
                         "from counters_collection").fetchall()
    with open(path, newline="") as f:
        rows = list(csv.DictReader(f))
    if not rows:
        return []
    key = lambda *c: next((k for k in rows[0] if k.lower() in c), None)
    kname, cname, cval = key("kernel_name"), key("counter_name"), key("counter_value")
    did, grid = key("dispatch_id", "correlation_id"), key("grid_size")
    return [(r[did], r[kname], int(r[grid]) if grid else 0, r[cname], float(r[cval])) for r in rows]


_EPI = re.compile(r"k_q([12])_apply<(float|double), (\d), (\d)")


def pmc(path: str, copy_mib: float = 0.0) -> str:
    rows = _pmc_rows(path)
    if not rows:
        return "no rows"
    per = {}
    for did, name, grid, cn, v in rows:
        d = per.setdefault(did, {"name": name, "grid": grid})
        d[cn] = d.get(cn, 0.0) + float(v)
    counters = sorted({r[3] for r in rows})
    out = ["counters: %s, %d dispatches" % (", ".join(counters), len(per))]
    factor = {}
    if copy_mib > 0:
        copies = [d for d in per.values() if "k_stream_copy" in d["name"] or "elementwise" in d["name"].lower()]
        if copies:
            for c in counters:
                best = max(copies, key=lambda d: d.get(c, 0.0))
                factor[c] = copy_mib * (1 << 20) / max(best.get(c, 0.0), 1e-30)
                out.append("copy calibration %s: %.1f counter units for %.0f MiB -> %.4f B per counter unit" % (
                    c, best.get(c, 0.0), copy_mib, factor[c]))
    cls = {}
    for d in per.values():
        m = _EPI.search(d["name"])
        if not m:
            continue
        k = "%s epi %s grid %d" % (apply_class(d["name"]), m.group(4), d["grid"])
        a = cls.setdefault(k, {"n": 0})
        a["n"] += 1
        for c in counters:
            a[c] = a.get(c, 0.0) + d.get(c, 0.0)
    out += ["", "| class, epilogue, grid | dispatches | " + " | ".join("%s units/dispatch" % c for c in counters) +
            "".join(" | %s MB/dispatch (calibrated)" % c for c in counters if c in factor) + " |",
            "|---|---|" + "---|" * (len(counters) + len(factor))]
    for k, a in sorted(cls.items()):
        row = "| %s | %d | " % (k, a["n"]) + " | ".join("%.1f" % (a[c] / a["n"]) for c in counters)
        row += "".join(" | %.3f" % (a[c] / a["n"] * factor[c] / 1e6) for c in counters if c in factor)
        out.append(row + " |")
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "pmc":
        print(pmc(sys.argv[2], float(sys.argv[3]) if len(sys.argv) > 3 else 0.0))
    elif len(sys.argv) >= 3 and sys.argv[1] == "trace":
        print(summarise(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 40))
    else:
        print(__doc__)
        sys.exit(2)
