"""Summaries of rocprofv3 output for the xmgn kernels.

  python -m paper_2411_17164_amd.profiling stats <rocprof output dir>
      per-kernel table from the --kernel-trace --stats CSV
  python -m paper_2411_17164_amd.profiling traffic --fetch <dir> --write <dir>
      --kernel <name substring> --calib <name substring> --calib-bytes <B>
      --workload <name> --out <json>
      HBM bytes per launch of a kernel from two --pmc runs (FETCH_SIZE, then
      WRITE_SIZE, KiB per dispatch), each scaled by what the same counter
      reads for a plain copy kernel of known size in the same process.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys
from collections import defaultdict


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[-1]


def demangle(name: str) -> str:
    """Readable name for this library's kernels, whose template arguments
    are only bf16, float and integer literals: _ZN4xmgn<len><name>I...E."""
    import re
    m = re.match(r"_ZN4xmgn(\d+)", name)
    if not m:
        return name
    i = m.end()
    kname = name[i:i + int(m.group(1))]
    i += int(m.group(1))
    if i >= len(name) or name[i] != "I":
        return kname
    i += 1
    args = []
    while i < len(name) and name[i] != "E":
        if name.startswith("DF16b", i):
            args.append("bf16")
            i += 5
        elif name[i] == "f":
            args.append("float")
            i += 1
        elif name[i] == "L":
            j = name.index("E", i)
            args.append(name[i + 2:j].replace("n", "-"))
            i = j + 1
        else:
            return name
    return f"{kname}<{', '.join(args)}>"


def short(name: str) -> str:
    """Demangled kernel name with its template arguments, without the
    namespace and the parameter list."""
    n = demangle(name)
    for tok in ("void ", "xmgn::"):
        n = n.replace(tok, "")
    return n.split("(")[0]


def stats(d: str):
    """[(kernel, calls, total ms, avg us, %)] from the --stats CSV, or from
    the kernel trace (rocpd2csv export) when no stats file exists."""
    rows = []
    try:
        path = _find(d, "kernel_stats.csv")
    except FileNotFoundError:
        path = None
    if path:
        with open(path) as f:
            for r in csv.DictReader(f):
                rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
                             float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    else:
        acc = defaultdict(lambda: [0, 0.0])
        with open(_find(d, "kernel_trace.csv")) as f:
            for r in csv.DictReader(f):
                a = acc[r["Kernel_Name"]]
                a[0] += 1
                a[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        tot = sum(v[1] for v in acc.values()) or 1.0
        rows = [(k, c, t, t / c * 1e3, 100.0 * t / tot) for k, (c, t) in acc.items()]
    rows.sort(key=lambda x: -x[2])
    return rows


def _counter_rows(d: str):
    try:
        path = _find(d, "counter_collection.csv")
    except FileNotFoundError:
        path = _find(d, "counter_collection_trace.csv")
    with open(path) as f:
        yield from csv.DictReader(f)


def counters(d: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter."""
    out = defaultdict(list)
    for r in _counter_rows(d):
        if r.get("Counter_Name") == counter:
            out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return out


def resources(d: str):
    """{kernel name: (VGPRs, AGPRs, SGPRs, LDS bytes, scratch bytes, workgroup size)}."""
    out = {}
    for r in _counter_rows(d):
        out[r["Kernel_Name"]] = tuple(int(float(r.get(k) or 0)) for k in (
            "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "LDS_Block_Size", "Scratch_Size", "Workgroup_Size"))
    return out


def _match(table, sub, largest=False):
    """Mean counter value over the dispatches of kernels whose name contains
    `sub` (or the largest one: a runtime copy kernel also serves small
    copies, and the calibration copy is the biggest of the run)."""
    names = [k for k in table if sub in k]
    if not names:
        raise KeyError(f"no kernel matching {sub!r}")
    vals = [v for k in names for v in table[k]]
    if largest:
        return max(vals), 1, names
    return sum(vals) / len(vals), len(vals), names


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--top", type=int, default=25)
    s.add_argument("--resources", default=None, help="a --pmc output dir: add register/LDS columns")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--calib", required=True)
    t.add_argument("--calib-bytes", type=float, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--source-hash", required=True)
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        rows = stats(a.dir)
        res = resources(a.resources) if a.resources else {}
        extra = " VGPR | AGPR | LDS B | scratch B | WG |" if res else ""
        print("| kernel | calls | total ms | avg us | % |" + extra)
        print("|---|---|---|---|---|" + ("---|" * 5 if res else ""))
        for name, calls, tot, avg, pct in rows[: a.top]:
            r = res.get(name)
            tail = (" " + " | ".join(str(r[i]) for i in (0, 1, 3, 4, 5)) + " |") if r else (" | | | | |" if res else "")
            print(f"| {short(name)[:100]} | {calls} | {tot:.3f} | {avg:.1f} | {pct:.2f} |{tail}")
        return 0
    fetch = counters(a.fetch, "FETCH_SIZE")
    write = counters(a.write, "WRITE_SIZE")
    cf, _, _ = _match(fetch, a.calib, largest=True)
    cw, _, _ = _match(write, a.calib, largest=True)
    kf, nf, names = _match(fetch, a.kernel)
    kw, nw, _ = _match(write, a.kernel)
    sf = a.calib_bytes / (cf * 1024.0)
    sw = a.calib_bytes / (cw * 1024.0)
    rec = {"kernel": a.kernel, "workload": a.workload, "source_hash": a.source_hash,
           "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw, "dispatches": [nf, nw],
           "calib_fetch_kib": cf, "calib_write_kib": cw, "calib_bytes": a.calib_bytes,
           "scale_fetch": sf, "scale_write": sw,
           "bytes_per_launch": kf * 1024.0 * sf + kw * 1024.0 * sw, "kernel_names": names[:4]}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
