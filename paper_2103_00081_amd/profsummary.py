"""Summarise rocprofv3 output per kernel.

Usage:
  python -m paper_2103_00081_amd.profsummary trace <run_results.db> [top]
      total device time, launches, average / minimum duration, grid size,
      VGPR count and scratch bytes per kernel (heaviest first), then the
      fine-level operator kernels grouped by (field, precision).
  python -m paper_2103_00081_amd.profsummary traffic <fetch.db> <write.db> <copy_mib>
      FETCH_SIZE + WRITE_SIZE bytes per launch of each operator class with
      the store epilogue, scaled by the counts of the library's plain copy of
      copy_mib MiB, with the hash of the operator sources they were taken on
      (the lines the benchmark reads).
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

# operator kernels: k_q1_pressure<T, EPI, ...>, k_q1_heat<T, EPI, ...>,
# k_q2_apply<T, FIELD, EPI, ...>
_Q1 = re.compile(r"k_q1_(pressure|heat)<(float|double), (\d)")
_Q2 = re.compile(r"k_q2_apply<(float|double), (\d), (\d)")


def apply_info(name: str):
    """(class, epilogue) of an operator kernel name, or None."""
    m = _Q1.search(name)
    if m:
        prec = "FP64" if m.group(2) == "double" else "FP32"
        return "Q1 %s apply %s" % (m.group(1), prec), m.group(3)
    m = _Q2.search(name)
    if m:
        prec = "FP64" if m.group(1) == "double" else "FP32"
        return "Q2 %s apply %s" % ("pressure" if m.group(2) == "0" else "heat", prec), m.group(3)
    return None


def short_name(name: str) -> str:
    s = name.replace("(anonymous namespace)::", "").split("(")[0]
    return re.sub(r"\s+", " ", s)


def apply_class(name: str):
    i = apply_info(name)
    return i[0] if i else None


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
        info = apply_info(d["name"])
        if not info:
            continue
        k = "%s epi %s grid %d" % (info[0], info[1], d["grid"])
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


def kernel_source_hash(root: str) -> str:
    """First 16 hex digits of the SHA-256 of the Q1 operator sources (the
    benchmark accepts a counter summary only for the source it was taken on)."""
    import hashlib
    import os
    src = [os.path.join(root, "paper_2103_00081_amd", "csrc", f) for f in ("op_q1.hip", "dev_util.h", "common.h")]
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in src)).hexdigest()[:16]


def traffic(fetch_db: str, write_db: str, copy_mib: float) -> str:
    """HBM-side bytes per launch of each operator class with the store
    epilogue: FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter
    reads for the library's plain copy of copy_mib MiB."""
    import os
    out = []
    per_class = {}
    for path, cname in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        per = {}
        for did, name, grid, cn, v in _pmc_rows(path):
            if cn != cname:
                continue
            d = per.setdefault(did, {"name": name, "grid": grid, "v": 0.0})
            d["v"] += float(v)
        copies = [d for d in per.values() if "k_stream_copy" in d["name"]]
        unit = copy_mib * (1 << 20) / max(max(d["v"] for d in copies), 1e-30)
        out.append("%s: %.4f B per counter unit (copy of %.0f MiB)" % (cname, unit, copy_mib))
        for d in per.values():
            info = apply_info(d["name"])
            if not info or info[1] != "0":
                continue
            a = per_class.setdefault(info[0], {}).setdefault(cname, [])
            a.append(d["v"] * unit)
    out.append("")
    out.append("| class | launches | FETCH MB | WRITE MB | total MB |")
    out.append("|---|---|---|---|---|")
    lines = []
    for k, c in sorted(per_class.items()):
        f = sum(c.get("FETCH_SIZE", [0])) / max(1, len(c.get("FETCH_SIZE", [1])))
        w = sum(c.get("WRITE_SIZE", [0])) / max(1, len(c.get("WRITE_SIZE", [1])))
        out.append("| %s | %d | %.2f | %.2f | %.2f |" % (k, len(c.get("FETCH_SIZE", [])), f / 1e6, w / 1e6,
                                                       (f + w) / 1e6))
        lines.append("traffic_bytes_per_launch %s %.0f" % (k, f + w))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out += ["", "kernel_source_sha256_16 %s" % kernel_source_hash(root)] + lines
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "pmc":
        print(pmc(sys.argv[2], float(sys.argv[3]) if len(sys.argv) > 3 else 0.0))
    elif len(sys.argv) >= 5 and sys.argv[1] == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], float(sys.argv[4])))
    elif len(sys.argv) >= 3 and sys.argv[1] == "trace":
        print(summarise(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 40))
    else:
        print(__doc__)
        sys.exit(2)
