"""Short text summaries of rocprofv3 output, for the committed profiles.

``trace``: the kernel-trace statistics (``*_kernel_stats.csv`` of a
``rocprofv3 --kernel-trace --stats --output-format csv`` run) as a table of
calls, average, minimum and total time per kernel.

``counters``: per kernel, the mean of each counter of one or more counter
runs (``rocprofv3 --pmc ...``, CSV output) over the kernel's dispatches.

``traffic``: HBM bytes per launch of one kernel from two counter runs
(``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``, CSV output), each
scaled by what the same counter reads for a plain device copy of known size
in the same run (the largest copy kernel's dispatch), with the SHA-256 of the
kernel's sources so that a reader can tell whether the figures still apply.

    python -m paper_1903_11785_amd.profile_summary trace DIR --command "..." > profiles/X.txt
    python -m paper_1903_11785_amd.profile_summary traffic FETCH_DIR WRITE_DIR \\
        --kernel carve_frame_kernel --sources a.hip b.h --copy-mib 256 \\
        --workload "..." --command "..." > profiles/X_traffic.json
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _one(pattern: str, d: str) -> str:
    fs = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not fs:
        raise SystemExit(f"no {pattern} under {d}")
    return fs[0]


def short_name(name: str) -> str:
    """The kernel's name without its parameter list (template arguments kept)."""
    depth, out = 0, []
    for ch in name:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).replace("void ", "").strip()


def trace(d: str, command: str, top: int, first: int = 0, first_kernels=()) -> str:
    rows = list(csv.DictReader(open(_one("*kernel_stats.csv", d))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# kernel trace: {command}", "",
             f"{'calls':>6} {'avg_us':>9} {'min_us':>9} {'total_us':>10}  kernel"]
    for r in rows[:top]:
        lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['MinNs']) / 1e3:9.2f} {float(r['TotalDurationNs']) / 1e3:10.1f}  "
                     f"{short_name(r['Name'])}")
    if first and first_kernels:
        # the first dispatches of the named kernels (a leg that runs first, e.g.
        # the eager frames whose kernel events a benchmark reads)
        disp = list(csv.DictReader(open(_one("*kernel_trace.csv", d))))
        disp.sort(key=lambda r: int(r["Start_Timestamp"]))
        lines += ["", f"# the first {first} dispatches of each of these kernels", "",
                  f"{'calls':>6} {'avg_us':>9} {'min_us':>9} {'max_us':>9}  kernel"]
        for k in first_kernels:
            ds = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                  for r in disp if short_name(r["Kernel_Name"]) == k][:first]
            if ds:
                lines.append(f"{len(ds):6d} {sum(ds) / len(ds):9.2f} {min(ds):9.2f} "
                             f"{max(ds):9.2f}  {k}")
    return "\n".join(lines) + "\n"


def _counter_rows(d: str, counter: str):
    """(dispatch id, kernel name, value) per dispatch for one counter."""
    path = _one("*counter_collection.csv", d)
    per = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", counter) != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        name = r.get("Kernel_Name", "")
        v = float(r["Counter_Value"])
        if key in per:
            per[key] = (name, per[key][1] + v)      # summed over instances
        else:
            per[key] = (name, v)
    return [(k, n, v) for k, (n, v) in per.items()]


def _kernel_mean(rows, kernel: str):
    """Mean over the dispatches whose short name (template arguments kept) is
    `kernel`, or that contain it as a name when it has no template arguments."""
    if "<" in kernel:
        vals = [v for _, n, v in rows if short_name(n) == kernel]
    else:
        vals = [v for _, n, v in rows if re.search(rf"\b{re.escape(kernel)}\b", n)]
    if not vals:
        raise SystemExit(f"no dispatch of {kernel}")
    return sum(vals) / len(vals), len(vals)


def _copy_value(rows):
    """The counter of the plain device copy: the largest dispatch of the HIP
    runtime's buffer copy (a device-to-device tensor copy launches it)."""
    vals = [v for _, n, v in rows if "copyBuffer" in n]
    if not vals:
        raise SystemExit("no copy dispatch for the reference")
    return max(vals)


def counters(dirs, kernels, command: str) -> str:
    """Per kernel, the mean of every counter over its dispatches, from one or
    more counter runs (each a rocprofv3 --pmc run with CSV output)."""
    per = {}
    for d in dirs:
        path = _one("*counter_collection.csv", d)
        acc = {}
        names = {}
        for r in csv.DictReader(open(path)):
            key = (r.get("Dispatch_Id"), r["Counter_Name"])
            acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
            names[r.get("Dispatch_Id")] = short_name(r["Kernel_Name"])
        for (did, cn), v in acc.items():
            per.setdefault(names[did], {}).setdefault(cn, []).append(v)
    lines = [f"# counters: {command}", "",
             "kernel | counter | mean per dispatch | dispatches"]
    for k in kernels:
        for cn, vs in sorted(per.get(k, {}).items()):
            lines.append(f"{k} | {cn} | {sum(vs) / len(vs):.6g} | {len(vs)}")
    return "\n".join(lines) + "\n"


def traffic(fetch_dir, write_dir, kernel, sources, copy_mib, workload, command) -> dict:
    """kernel: one short name, or several joined by ' + ' (a call of several
    kernels: the sum of their means)."""
    fr, wr = _counter_rows(fetch_dir, "FETCH_SIZE"), _counter_rows(write_dir, "WRITE_SIZE")
    f_kib = w_kib = 0.0
    nf, nw = [], []
    for k in kernel.split(" + "):
        f, n1 = _kernel_mean(fr, k)
        w, n2 = _kernel_mean(wr, k)
        f_kib += f
        w_kib += w
        nf.append(n1)
        nw.append(n2)
    nf = nf[0] if len(nf) == 1 else nf
    nw = nw[0] if len(nw) == 1 else nw
    ref_kib = copy_mib * 1024.0
    f_copy, w_copy = _copy_value(fr), _copy_value(wr)
    f_scale, w_scale = ref_kib / f_copy, ref_kib / w_copy
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return {
        "kernel": kernel,
        "workload": workload,
        "sources": list(sources),
        "source_sha256": h.hexdigest(),
        "fetch_kib_per_launch": f_kib,
        "write_kib_per_launch": w_kib,
        "dispatches": [nf, nw],
        "reference_copy_mib": copy_mib,
        "reference_fetch_kib": f_copy,
        "reference_write_kib": w_copy,
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "traffic_bytes_per_launch": (f_kib * f_scale + w_kib * w_scale) * 1024.0,
        "note": "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what they read for a "
                f"plain {copy_mib} MiB device copy in the same run",
        "command": command,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--command", required=True)
    t.add_argument("--top", type=int, default=30)
    t.add_argument("--first", type=int, default=0,
                   help="also the statistics of the first N dispatches of --first-kernels")
    t.add_argument("--first-kernels", nargs="*", default=[])
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--kernel", required=True)
    c.add_argument("--sources", nargs="+", required=True)
    c.add_argument("--copy-mib", type=int, default=256)
    c.add_argument("--workload", required=True)
    c.add_argument("--command", required=True)
    q = sub.add_parser("counters")
    q.add_argument("dirs", nargs="+")
    q.add_argument("--kernels", nargs="+", required=True)
    q.add_argument("--command", required=True)
    a = ap.parse_args()
    if a.what == "counters":
        sys.stdout.write(counters(a.dirs, a.kernels, a.command))
    elif a.what == "trace":
        sys.stdout.write(trace(a.dir, a.command, a.top, a.first, a.first_kernels))
    else:
        json.dump(traffic(a.fetch_dir, a.write_dir, a.kernel, a.sources, a.copy_mib, a.workload,
                          a.command), sys.stdout, indent=1)
        sys.stdout.write("\n")


if __name__ == "__main__":
    main()
