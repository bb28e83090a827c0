"""Summaries of rocprofv3 output for the committed profile records.

    python -m paper_2406_13651_amd.profsum stats KERNEL_STATS_CSV [--top N]
        markdown table of a --kernel-trace --stats run (kernel, calls, avg,
        min, max, share of GPU time)

    python -m paper_2406_13651_amd.profsum phases [--trace TRACE_CSV] [--counters PMC_CSV]
        CNN kernels of a learned-workload run split into training and
        evaluation (at the first CLAMP iteration kernel): mean durations,
        mean counter values

    python -m paper_2406_13651_amd.profsum cnn --fetch FETCH_CSV --write WRITE_CSV --probe-mib M [--out JSON]
        HBM bytes of one CNN prior application (the learned workload's
        evaluation phase), stored for bench.py's learned line

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


CNN_KERNELS = (r"k_conv", r"k_wgrad", r"k_pack\(", r"k_grad_clip\(", r"k_grad_sq\(", r"k_prep_", r"k_adam\(", r"k_loss",
               # the U-Net's own kernels (pooling, transposed convolutions, batch normalisation)
               r"k_upconv", r"k_pool2", r"k_chan_", r"k_affine<", r"k_fold_bn\(", r"k_sum_blocks\(")


def _phase_start(ids_names):
    """Index of the first CLAMP iteration kernel in dispatch order: kernels
    before it belong to training, from it on to the evaluation."""
    return next((i for i, (_, name) in enumerate(ids_names) if re.search(r"k_row_grad<|k_row_upd_mann<", name)),
                len(ids_names))


def _short(name):
    return name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace("clampk::", "")


def phases_trace(path, top=14):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    start = _phase_start([(0, r["Kernel_Name"]) for r in rows])
    acc = collections.defaultdict(list)
    for i, r in enumerate(rows):
        if any(re.search(p, r["Kernel_Name"]) for p in CNN_KERNELS):
            ph = "evaluation" if i >= start else "training"
            acc[(_short(r["Kernel_Name"]), ph)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = ["| kernel | phase | launches | avg us | total us |", "|---|---|---:|---:|---:|"]
    for (k, ph), v in sorted(acc.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append("| `%s` | %s | %d | %.1f | %.0f |" % (k, ph, len(v), sum(v) / len(v), sum(v)))
    return "\n".join(out)


def phases_counters(path, counters):
    rows = list(csv.DictReader(open(path)))
    disp = collections.OrderedDict()
    for r in rows:
        disp.setdefault(int(r["Dispatch_Id"]), r["Kernel_Name"])
    order = sorted(disp.items())
    start_id = order[_phase_start(order)][0] if _phase_start(order) < len(order) else None
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        if any(re.search(p, r["Kernel_Name"]) for p in CNN_KERNELS):
            ph = "evaluation" if start_id is not None and int(r["Dispatch_Id"]) >= start_id else "training"
            acc[(_short(r["Kernel_Name"]), ph)][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = ["| kernel | phase | " + " | ".join(counters) + " |", "|---|---|" + "---:|" * len(counters)]
    for (k, ph), d in sorted(acc.items()):
        out.append("| `%s` | %s | " % (k, ph) + " | ".join(
            "%.3g" % (sum(d[c]) / len(d[c])) if d.get(c) else "" for c in counters) + " |")
    return "\n".join(out)


CNN_APPLY = (r"k_pack\(", r"k_conv_first\(", r"k_conv<", r"k_conv_final\(", r"k_sum_partial\(", r"k_mean_final\(")


def cnn_traffic(fetch_csv, write_csv, probe_mib):
    """HBM bytes of one CNN prior application in the evaluation phase of a
    learned-workload run: every CNN kernel dispatched after the first CLAMP
    iteration kernel, summed and divided by the number of applications (one
    k_conv_final each)."""
    probe_bytes = probe_mib * (1 << 20)
    out = {}
    for path, counter, key in ((fetch_csv, "FETCH_SIZE", "read_bytes"), (write_csv, "WRITE_SIZE", "write_bytes")):
        rows = sorted(_counter_rows(path, counter))
        scale = probe_bytes / _probe(rows, probe_bytes)
        start = next((i for i, r in enumerate(rows) if re.search(r"k_row_grad<|k_row_upd_mann<", r[1])), None)
        if start is None:
            raise SystemExit("no CLAMP iteration kernel in " + path)
        ev = [r for r in rows[start:] if any(re.search(p, r[1]) for p in CNN_APPLY)]
        n = sum(1 for r in ev if "k_conv_final" in r[1])
        if n == 0:
            raise SystemExit("no CNN application after the first CLAMP iteration kernel in " + path)
        out[key] = sum(r[3] for r in ev) * scale / n
        out["applications"] = n
    return out


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
    t.add_argument("--shape", type=float, nargs=5, metavar=("NX", "NY", "NZ", "LOOKS", "RADIUS"),
                   help="workload of the runs (circular pupil, Gaussian prior, fused Mann step): adds the "
                        "algorithmic bytes of each stage and the counter / algorithmic ratio")
    t.add_argument("--stats", help="kernel-trace stats CSV of the same workload: adds the average duration and "
                                   "the algorithmic GB/s")
    t.add_argument("--out")
    ph = sub.add_parser("phases")
    ph.add_argument("--trace", help="kernel-trace CSV (kernel_trace.csv) of a learned-workload run")
    ph.add_argument("--top", type=int, default=14, help="rows of the kernel-duration table")
    ph.add_argument("--counters", help="--pmc counter CSV of a learned-workload run")
    ph.add_argument("--names", nargs="*", default=["SQ_VALU_MFMA_BUSY_CYCLES", "SQ_INSTS_LDS",
                                                   "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_LDS", "SQ_BUSY_CYCLES"])
    c = sub.add_parser("cnn")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--probe-mib", type=int, required=True)
    c.add_argument("--workload", default="cnn_apply_64x256x256")
    c.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "phases":
        if a.trace:
            print(phases_trace(a.trace, a.top))
        if a.counters:
            print(phases_counters(a.counters, a.names))
        return 0
    if a.cmd == "cnn":
        r = cnn_traffic(a.fetch, a.write, a.probe_mib)
        print("CNN application: %.1f MB read, %.1f MB written (mean of %d applications)"
              % (r["read_bytes"] / 1e6, r["write_bytes"] / 1e6, r["applications"]))
        if a.out:
            rec = json.load(open(a.out)) if os.path.exists(a.out) else {}
            rec[a.workload] = {"source_sha256": kernel_source_hash("cnn"), "read_bytes": r["read_bytes"],
                               "write_bytes": r["write_bytes"],
                               "launches": "first (from the fp32 volume), six middle and output convolutions, scale reductions"}
            with open(a.out, "w") as f:
                json.dump(rec, f, indent=1)
                f.write("\n")
        return 0
    if a.cmd == "stats":
        print(stats_table(a.csv, a.top))
        return 0
    per, fk, wk = traffic(a.fetch, a.write, a.probe_mib, a.skip_first)
    print("calibration: bytes = FETCH_SIZE x %.3f KiB, WRITE_SIZE x %.3f KiB" % (fk, wk))
    alg = {}
    if a.shape:
        from .perf import stage_bytes
        nx, ny, nz, looks, radius = int(a.shape[0]), int(a.shape[1]), int(a.shape[2]), int(a.shape[3]), a.shape[4]
        # the circular pupil of the plan: ku^2 + kv^2 <= R^2 in signed DFT indices
        sig = lambda k, n: k - n if 2 * k >= n else k  # noqa: E731
        cols = [sum(1 for u in range(ny) if sig(u, ny) ** 2 + sig(v, nx) ** 2 <= radius ** 2) for v in range(nx)]
        P, B = sum(cols), sum(1 for c in cols if c > 0)
        alg = stage_bytes(nx, ny, nz, looks, P, B, looks + 1, fused=True)
    avg_us = {}
    if a.stats:
        for r in csv.DictReader(open(a.stats)):
            st = stage_of(r["Name"])
            if st is not None:
                avg_us[st] = avg_us.get(st, 0.0) + float(r["AverageNs"]) / 1e3
    print("| stage | kernels | read MB | written MB | counter MB | algorithmic MB | counter / algorithmic "
          "| avg us | algorithmic GB/s |\n|---|---|---:|---:|---:|---:|---:|---:|---:|")
    for st, e in sorted(per.items(), key=lambda kv: -(kv[1]["read_bytes"] + kv[1]["write_bytes"])):
        tot = e["read_bytes"] + e["write_bytes"]
        ab = alg.get(st)
        us = avg_us.get(st)
        print("| %s | %s | %.1f | %.1f | %.1f | %s | %s | %s | %s |" % (
            st, ", ".join("`%s`" % k.split("(")[0].replace("void ", "").replace("clampk::", "") for k in e["kernels"]),
            e["read_bytes"] / 1e6, e["write_bytes"] / 1e6, tot / 1e6,
            "%.1f" % (ab / 1e6) if ab else "", "%.2f" % (tot / ab) if ab else "",
            "%.1f" % us if us else "", "%.0f" % (ab / (us * 1e-6) / 1e9) if ab and us else ""))
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
