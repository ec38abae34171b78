"""Summaries of rocprofv3 CSV output for the library's kernels.

    python -m paper_1401_7824_amd.profiling trace RUN_kernel_trace.csv
    python -m paper_1401_7824_amd.profiling counters FETCH.csv WRITE.csv \\
        --workload rd2d --kernel 'k_rows_rbgs_restrict<double, false, 0>' --workgroups 1216 \\
        --alg-bytes 27205664 [--update profiles/traffic.json]

`trace` prints the median duration per (kernel, workgroup count) -- the
workgroup count identifies the multigrid level.  `counters` reads one
FETCH_SIZE and one WRITE_SIZE counter run (each taken in a run of its own),
calibrates both against the plain 512 MiB device copy that bench.py
--calib-copy adds (FETCH_SIZE and WRITE_SIZE are in KiB; the copy reads and
writes 512 MiB), and reports the HBM bytes per launch of one kernel beside
its algorithmic bytes; --update stores the figure for bench.py, keyed by
workload and kernel, together with a hash of the kernel sources so that a
later change to them makes bench.py report the figure as stale (null).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# sources of the multigrid kernels; counter figures taken before a change to
# any of them are stale
TRAFFIC_SOURCES = ("paper_1401_7824_amd/csrc/mg_tiles.hip", "paper_1401_7824_amd/csrc/mg_device.h",
                   "paper_1401_7824_amd/csrc/mg_march.h", "paper_1401_7824_amd/csrc/tile_common.h",
                   "paper_1401_7824_amd/csrc/rows2d.h", "paper_1401_7824_amd/csrc/tailc.h")
COPY_KIB = 512 * 1024


def sources_sha256(root: str = ROOT) -> str:
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _short(name: str) -> str:
    for pre in ("void isdc::(anonymous namespace)::", "isdc::(anonymous namespace)::"):
        name = name.replace(pre, "")
    return name.split("(")[0]


def _groups(rows):
    return int(rows["Grid_Size"]) // int(rows["Workgroup_Size"])


def trace_table(path: str):
    """[(kernel, workgroups, launches, median_us, total_ms)] sorted by total time."""
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        wg = (int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])) // int(r["Workgroup_Size_X"])
        d[(_short(r["Kernel_Name"]), wg)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = []
    for (k, wg), v in d.items():
        out.append((k, wg, len(v), statistics.median(v) / 1e3, sum(v) / 1e6))
    out.sort(key=lambda t: -t[4])
    return out


def counter_medians(path: str):
    """{(kernel, workgroups): [values]} of one counter run."""
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[(_short(r["Kernel_Name"]), _groups(r))].append(float(r["Counter_Value"]))
    return d


def calibration(d) -> float:
    """Counter KiB of the 512 MiB copy (the largest copy launch of the run)."""
    vals = [v for (k, _), vs in d.items() if "copyBuffer" in k for v in vs]
    if not vals:
        raise SystemExit("no device copy in this counter run (bench.py --calib-copy adds one)")
    return max(vals)


def counters(fetch_csv: str, write_csv: str, kernel: str, workgroups: int):
    fe, wr = counter_medians(fetch_csv), counter_medians(write_csv)
    f_scale = COPY_KIB / calibration(fe)
    w_scale = COPY_KIB / calibration(wr)
    key = (kernel, workgroups)
    if key not in fe or key not in wr:
        raise SystemExit(f"kernel {kernel!r} with {workgroups} workgroups not in the counter runs")
    f_kib, w_kib = statistics.median(fe[key]), statistics.median(wr[key])
    return dict(fetch_kib=f_kib, write_kib=w_kib, fetch_scale=f_scale, write_scale=w_scale,
                bytes_per_launch=(f_kib * f_scale + w_kib * w_scale) * 1024.0, launches=len(fe[key]))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--top", type=int, default=30)
    c = sub.add_parser("counters")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("--workload", required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--workgroups", type=int, required=True)
    c.add_argument("--alg-bytes", type=float, required=True)
    c.add_argument("--update")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        rows = trace_table(a.csv)
        tot = sum(r[4] for r in rows)
        print("| kernel | workgroups | launches | median us | % of kernel time |")
        print("|---|---:|---:|---:|---:|")
        for k, wg, n, med, ms in rows[: a.top]:
            print(f"| `{k}` | {wg} | {n} | {med:.2f} | {100 * ms / tot:.1f} |")
        print(f"\ntotal kernel time {tot:.2f} ms")
        return
    rec = counters(a.fetch_csv, a.write_csv, a.kernel, a.workgroups)
    rec.update(workload=a.workload, alg_bytes=a.alg_bytes, ratio=rec["bytes_per_launch"] / a.alg_bytes,
               sources_sha256=sources_sha256())
    print(json.dumps(rec, indent=1))
    if a.update:
        db = json.load(open(a.update)) if os.path.exists(a.update) else {}
        db[f"{a.workload}:{a.kernel.replace(', ', ',')}"] = rec
        with open(a.update, "w") as fh:
            json.dump(db, fh, indent=1)


if __name__ == "__main__":
    main()
