"""Summaries of rocprofv3 output for one kernel family (the range-finder sweeps
by default), written to profiles/.

    python -m paper_2508_08873_amd.prof_summary --name NAME --command CMD \\
        --stats DIR/kt_kernel_stats.csv --calls N \\
        [--fetch DIR/..._counter_collection.csv --write DIR/..._counter_collection.csv \\
         --fetch-calls M --calib-fetch DIR/... --calib-write DIR/... --calib-bytes B]
        [--mfma DIR/..._counter_collection.csv --mfma-calls M] [--kernel PATTERNS --label TEXT] [--bench bench.json]

A range-finder sweep (one library call: 32 implicit-Euler steps of 3200
right-hand sides) is one k_sweep launch, or, on factors with the UL set, two
k_sweep launches (the first and last substitutions) and 31 k_sweep_pair
launches.  --calls / --fetch-calls: the number of such calls in the traced /
counted command; time and bytes are reported per call.

Writes profiles/NAME.md (human-readable: per-kernel time table, HBM bytes per
sweep call, the calibration factors) and profiles/NAME.json (the figures
bench.py reads for ``roofline.traffic``), both stamped with a hash of the
sweep's sources: bench.py reports the traffic only while the sources still
hash to the same value.

HBM bytes: FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is scaled
by (bytes a plain device copy of known size moves) / (what the same counter
reads for that copy).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
# the sweep kernels, their launch logic and the structures they read (the
# tile contents that csrc/factor.hip writes do not change what a sweep moves)
SWEEP_SOURCES = ["csrc/sweep.hip", "csrc/lrpr_internal.h", "csrc/tile_ops.h", "csrc/api_core.cpp"]


def sweep_source_hash() -> str:
    h = hashlib.sha1()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter(path, matches):
    vals = []
    for r in csv.DictReader(open(path)):
        if any(m in r["Kernel_Name"] for m in matches):
            vals.append(float(r["Counter_Value"]) * 1024.0)
    return vals


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", required=True)
    ap.add_argument("--command", required=True, help="the full command the figures come from")
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--calib-fetch")
    ap.add_argument("--calib-write")
    ap.add_argument("--calib-bytes", type=float, default=0.0)
    ap.add_argument("--calib-kernel", default="copyBuffer")
    ap.add_argument("--kernel", default="k_sweep<,k_sweep_pair<",
                    help="comma-separated substrings of the kernel names of a sweep (the default excludes "
                         "k_sweep_local, the partitioned block solves)")
    ap.add_argument("--calls", type=int, required=True, help="sweep calls in the traced command")
    ap.add_argument("--fetch-calls", type=int, default=0, help="sweep calls in each counter command")
    ap.add_argument("--mfma", help="counter collection of SQ_INSTS_VALU_MFMA_MOPS_F32/_F64, "
                                   "SQ_VALU_MFMA_BUSY_CYCLES and SQ_BUSY_CU_CYCLES")
    ap.add_argument("--mfma-calls", type=int, default=0, help="sweep calls in the MFMA counter command")
    ap.add_argument("--label", default="Range-finder sweeps", help="what the matched kernels are")
    ap.add_argument("--bench")
    args = ap.parse_args()

    rows = list(csv.DictReader(open(args.stats)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["# rocprofv3 summary: %s" % args.name, "", "Command:", "", "    " + args.command, "",
             "Kernel time (`--kernel-trace --stats`):", "",
             "| kernel | calls | total ms | avg ms | % |", "|---|---|---|---|---|"]
    for r in rows[:14]:
        name = r["Name"]
        if len(name) > 70:
            name = name[:67] + "..."
        lines.append("| `%s` | %s | %.2f | %.4f | %.1f |" % (name.replace("|", "/"), r["Calls"],
                                                           float(r["TotalDurationNs"]) / 1e6,
                                                           float(r["AverageNs"]) / 1e6,
                                                           100.0 * float(r["TotalDurationNs"]) / total))
    pats = [k for k in args.kernel.split(",") if k]
    sweep = [r for r in rows if any(k in r["Name"] for k in pats)]
    launches = sum(int(r["Calls"]) for r in sweep)
    per_call_ms = sum(float(r["TotalDurationNs"]) for r in sweep) / args.calls / 1e6
    out = {"name": args.name, "command": args.command, "kernel": args.kernel, "source_sha1": sweep_source_hash(),
           "sweep_calls": args.calls, "sweep_launches": launches, "sweep_ms_per_call": per_call_ms}
    lines += ["", "%s (kernels matching %s, all instantiations): %d launches in %d calls, "
              "%.3f ms per call." % (args.label, ", ".join("`%s`" % k for k in pats), launches, args.calls,
                                     per_call_ms)]
    if args.fetch and args.write and args.calib_fetch and args.calib_write and args.calib_bytes > 0:
        cf = _counter(args.calib_fetch, args.calib_kernel)
        cw = _counter(args.calib_write, args.calib_kernel)
        kf = args.calib_bytes / statistics.mean(cf)
        kw = args.calib_bytes / statistics.mean(cw)
        f = _counter(args.fetch, pats)
        w = _counter(args.write, pats)
        nc = args.fetch_calls or args.calls
        fb = sum(f) * kf / nc
        wb = sum(w) * kw / nc
        out.update({"calib_factor_fetch": kf, "calib_factor_write": kw, "fetch_bytes_per_sweep": fb,
                    "write_bytes_per_sweep": wb, "traffic_bytes_per_sweep": fb + wb,
                    "counted_dispatches": len(f), "counted_sweep_calls": nc})
        lines += ["", "HBM traffic (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`, separate runs of the same command):",
                  "",
                  "- copy calibration: a %.0f-byte device copy reads FETCH_SIZE x %.3f and WRITE_SIZE x %.3f of "
                  "the bytes it moves; the factors below undo that" % (args.calib_bytes, 1 / kf, 1 / kw),
                  "- factors: fetch x %.3f, write x %.3f" % (kf, kw),
                  "- per sweep call (%d dispatches over %d calls): fetch %.2f GB, write %.2f GB, total %.2f GB" %
                  (len(f), nc, fb / 1e9, wb / 1e9, (fb + wb) / 1e9)]
    if args.mfma:
        sums = {}
        for r in csv.DictReader(open(args.mfma)):
            if any(m in r["Kernel_Name"] for m in pats):
                sums[r["Counter_Name"]] = sums.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        nc = args.mfma_calls or args.calls
        f32 = sums.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) * 512.0 / nc
        f64 = sums.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512.0 / nc
        busy, cu = sums.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0), sums.get("SQ_BUSY_CU_CYCLES", 0.0)
        util = busy / (4.0 * cu) if cu > 0 else None
        out.update({"mfma_flops_f32_per_call": f32, "mfma_flops_f64_per_call": f64, "mfma_busy_frac": util})
        lines += ["", "Matrix cores (`--pmc SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_INSTS_VALU_MFMA_MOPS_F64 "
                  "SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CU_CYCLES`, a run of its own):", "",
                  "- MFMA flops per call (MOPS x 512): FP32 %.4g, FP64 %.4g" % (f32, f64),
                  "- MFMA busy cycles / (4 SIMDs x busy CU cycles): %s" % ("%.3f" % util if util is not None else "n/a")]
        if per_call_ms > 0:
            lines.append("- MFMA rate over the traced kernel time: FP32 %.1f TFLOP/s, FP64 %.1f TFLOP/s"
                         % (f32 / per_call_ms / 1e9, f64 / per_call_ms / 1e9))
    if args.bench:
        b = json.loads(open(args.bench).read().strip().splitlines()[-1])
        lines += ["", "Bench line of the same build:", "", "    " + json.dumps(b)]
    lines += ["", "Sweep sources hash (sha1 of %s): `%s`" % (", ".join(SWEEP_SOURCES), out["source_sha1"])]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", args.name + ".md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(os.path.join(ROOT, "profiles", args.name + ".json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote profiles/%s.md and .json" % args.name)


if __name__ == "__main__":
    main()
