"""Summarise rocprofv3 CSV output into the short text/JSON files kept in profiles/.

    python -m paper_1305_1183_amd.rocprof_summary --trace DIR --fetch DIR --write DIR \
        --copy-fetch DIR --copy-write DIR --copy-bytes B --out-dir profiles --tag NAME --cmd "..."

* kernel statistics (``*_kernel_stats.csv`` of ``--kernel-trace --stats``) are
  written as ``<tag>_kernel_stats.txt``;
* FETCH_SIZE / WRITE_SIZE (KiB per dispatch, ``--pmc`` runs) are averaged per
  kernel and scaled by the ratio of the copy kernel's true byte count to what
  the same counter reports for it; the result goes to ``pmc_summary.json``.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os


def _csv(d, suffix):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return list(csv.DictReader(open(files[0])))


def counter_means(d):
    agg = collections.defaultdict(list)
    for r in _csv(d, "_counter_collection.csv"):
        agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--out-dir", default="profiles")
    ap.add_argument("--tag", required=True)
    ap.add_argument("--pmc-out", default="pmc_summary.json")
    ap.add_argument("--pmc-match", default="kf_", help="kernels whose name contains this are kept")
    ap.add_argument("--by-grid", default="",
                    help="kernels whose name contains this are listed per grid size, from the dispatch trace")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--pmc-cmd", default="")
    a = ap.parse_args()
    os.makedirs(a.out_dir, exist_ok=True)
    if a.trace and a.by_grid:
        agg = collections.defaultdict(list)
        vg = {}
        for r in _csv(a.trace, "_kernel_trace.csv"):
            name = r["Kernel_Name"]
            if a.by_grid in name:
                name = "%s grid=%d" % (a.by_grid, int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"])))
                key = name if int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"])) >= 256 else a.by_grid + " grid<256"
            else:
                key = name.split("(")[0]
            agg[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
            vg[key] = r["VGPR_Count"]
        tot = sum(sum(v) for v in agg.values())
        lines = ["# rocprofv3 --kernel-trace (per dispatch, grouped by grid size): %s" % a.tag,
                 "# command: %s" % a.cmd,
                 "%-44s %7s %12s %10s %10s %6s %8s" % ("kernel", "calls", "avg_us", "min_us", "max_us", "vgpr", "pct")]
        for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
            lines.append("%-44s %7d %12.2f %10.2f %10.2f %6s %8.2f" % (k[:44], len(v), sum(v) / len(v), min(v), max(v),
                                                                     vg[k], 100.0 * sum(v) / tot))
        with open(os.path.join(a.out_dir, a.tag + "_kernel_stats.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
    elif a.trace:
        rows = _csv(a.trace, "_kernel_stats.csv")
        lines = ["# rocprofv3 --kernel-trace --stats: %s" % a.tag,
                 "# command: %s" % a.cmd,
                 "%-44s %6s %12s %10s %10s %10s" % ("kernel", "calls", "avg_us", "min_us", "max_us", "pct")]
        for r in rows:
            lines.append("%-44s %6s %12.2f %10.2f %10.2f %10s" % (
                r["Name"][:44], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                float(r["MaxNs"]) / 1e3, r["Percentage"]))
        with open(os.path.join(a.out_dir, a.tag + "_kernel_stats.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
    if a.fetch and a.write and a.copy_fetch and a.copy_write:
        fe, wr = counter_means(a.fetch), counter_means(a.write)
        cf, cw = counter_means(a.copy_fetch), counter_means(a.copy_write)
        copy_f = [v for (k, c), v in cf.items() if "kf_copy_f4_kernel" in k][0][0]
        copy_w = [v for (k, c), v in cw.items() if "kf_copy_f4_kernel" in k][0][0]
        sf = a.copy_bytes / (copy_f * 1024.0)
        sw = a.copy_bytes / (copy_w * 1024.0)
        kernels = {}
        for (k, c), (v, n) in fe.items():
            if c != "FETCH_SIZE" or a.pmc_match not in k:
                continue
            w = wr.get((k, "WRITE_SIZE"), (0.0, 0))[0]
            kernels[k] = {"fetch_kib": round(v, 1), "write_kib": round(w, 1), "dispatches": n,
                          "fetch_bytes_scaled": round(v * 1024 * sf), "write_bytes_scaled": round(w * 1024 * sw)}
        out = {"source": "rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE, separate runs, KiB per dispatch",
               "command": a.pmc_cmd,
               "calibration": {"copy_bytes_each_way": a.copy_bytes, "copy_fetch_kib": round(copy_f, 1),
                               "copy_write_kib": round(copy_w, 1), "fetch_scale": round(sf, 4),
                               "write_scale": round(sw, 4)},
               "kernels": kernels}
        path = os.path.join(a.out_dir, a.pmc_out)
        with open(path, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
