"""Summaries of rocprofv3 output for the committed profile records.

    python -m paper_2406_13651_amd.profsum stats KERNEL_STATS_CSV [--top N]
        markdown table of a --kernel-trace --stats run (kernel, calls, avg,
        min, max, share of GPU time)

    python -m paper_2406_13651_amd.profsum traffic --fetch FETCH_CSV --write WRITE_CSV
            --probe-mib M --workload NAME [--out JSON] [--skip-first K]
        HBM bytes per launch of each forward-path stage (each stage one
        launch per iteration) from two --pmc runs (FETCH_SIZE,
        then WRITE_SIZE, KiB per dispatch), scaled by what the same counters
        read for the M MiB device copy that `bench.py --copy-probe M` issues
        (the one __amd_rocclr_copyBuffer dispatch of that size); prints a
        markdown table and, with --out, stores the record that bench.py
        reports as roofline.traffic while the kernel sources still hash the
        same.

Stages are the library's timing stages; a kernel maps to its stage by name.
"""

from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
KERNEL_SOURCES = {
    "fwd": ("fft.hpp", "internal.h", "passes.hpp", "kernels.hip", "api.cpp"),
    "cnn": ("cnn.h", "cnn.hip", "cnn_api.cpp"),
}

# kernel name pattern -> timing stage (first match wins)
STAGE_OF = [
    (r"k_row_upd_mann", "row_update_mann"),
    (r"k_row_grad<", "row_grad"),
    (r"k_row<\d+, 3>|k_row<\d+, 4>", "row_update"),
    (r"k_col_inv_compact<", "col_inv"),
    (r"k_col_fwd<", "col_fwd"),
    (r"k_resid\(", "resid_update"),
    (r"k_gauss3d<", "prior_gauss"),
    (r"k_mace<|k_mace_final\(", "mace_step"),
    (r"k_gamma\(", "gamma"),
    (r"k_diag_after\(", "diag_after"),
]


def kernel_source_hash(group):
    """sha256 over the kernel sources of one group (forward path or CNN)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[group]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stage_of(kernel):
    for pat, st in STAGE_OF:
        if re.search(pat, kernel):
            return st
    return None


def stats_table(path, top=20):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg us | min us | max us | % |", "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"].replace("|", "\\|")
        if len(name) > 90:
            name = name[:87] + "..."
        out.append("| `%s` | %s | %.1f | %.1f | %.1f | %.1f |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    return "\n".join(out)


def _counter_rows(path, counter):
    """(dispatch id, kernel name, grid size, value) of one counter, summed
    over the instances the CSV lists for a dispatch."""
    acc = collections.OrderedDict()
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = int(r["Dispatch_Id"])
        if key not in acc:
            acc[key] = [r["Kernel_Name"], int(r["Grid_Size"]), 0.0]
        acc[key][2] += float(r["Counter_Value"])
    return [(k, v[0], v[1], v[2]) for k, v in acc.items()]


def _probe(rows, probe_bytes):
    """Counter value of the copy probe: the largest copyBuffer dispatch."""
    cands = [v for _, name, grid, v in rows if "copyBuffer" in name]
    if not cands:
        raise SystemExit("no __amd_rocclr_copyBuffer dispatch in the counter file")
    return max(cands)


def traffic(fetch_csv, write_csv, probe_mib, skip_first=1):
    probe_bytes = probe_mib * (1 << 20)
    fr, wr = _counter_rows(fetch_csv, "FETCH_SIZE"), _counter_rows(write_csv, "WRITE_SIZE")
    # a device copy of B bytes reads B and writes B
    f_scale = probe_bytes / _probe(fr, probe_bytes)
    w_scale = probe_bytes / _probe(wr, probe_bytes)
    per = {}
    for rows, key, scale in ((fr, "read_bytes", f_scale), (wr, "write_bytes", w_scale)):
        seen = collections.Counter()
        sums = collections.defaultdict(list)
        for _, name, _, v in rows:
            st = stage_of(name)
            if st is None:
                continue
            seen[name] += 1
            if seen[name] <= skip_first:  # the first launches (plan set-up, cold caches)
                continue
            sums[(st, name)].append(v * scale)
        for (st, name), vals in sums.items():
            e = per.setdefault(st, {"read_bytes": 0.0, "write_bytes": 0.0, "kernels": []})
            e[key] += sum(vals) / len(vals)
            if name not in e["kernels"]:
                e["kernels"].append(name)
    return per, f_scale / 1024.0, w_scale / 1024.0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=20)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--probe-mib", type=int, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--group", default="fwd", choices=("fwd",),
                   help="kernel source group whose hash the record carries (the forward path)")
    t.add_argument("--skip-first", type=int, default=1)
    t.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_table(a.csv, a.top))
        return 0
    per, fk, wk = traffic(a.fetch, a.write, a.probe_mib, a.skip_first)
    print("calibration: bytes = FETCH_SIZE x %.3f KiB, WRITE_SIZE x %.3f KiB" % (fk, wk))
    print("| stage | read MB | written MB | kernels |\n|---|---:|---:|---|")
    for st, e in sorted(per.items(), key=lambda kv: -(kv[1]["read_bytes"] + kv[1]["write_bytes"])):
        print("| %s | %.1f | %.1f | %s |" % (st, e["read_bytes"] / 1e6, e["write_bytes"] / 1e6,
                                             ", ".join("`%s`" % k.split("(")[0] for k in e["kernels"])))
    if a.out:
        rec = json.load(open(a.out)) if os.path.exists(a.out) else {}
        rec["note"] = ("HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs, scaled by a device-copy "
                       "probe; valid while the kernel sources hash to source_sha256")
        entry = {"source_sha256": kernel_source_hash(a.group),
                 "calibration_kib": {"fetch": round(fk, 4), "write": round(wk, 4), "probe_mib": a.probe_mib}}
        entry["stages"] = {st: {"read_bytes": e["read_bytes"], "write_bytes": e["write_bytes"]}
                           for st, e in per.items()}
        rec[a.workload] = entry
        with open(a.out, "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
