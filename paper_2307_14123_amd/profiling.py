"""Summaries of rocprofv3 output for the kernels of this library.

  python -m paper_2307_14123_amd.profiling stats <kernel_stats.csv> --command "<cmd>" --out <file.md>
      per-kernel launch counts and durations (from --kernel-trace --stats, csv output),
      grouped by the families bench.py reports
  python -m paper_2307_14123_amd.profiling hbm <fetch dir> <write dir> <kernel_stats.csv> --command "<cmd>" --out <file.md>
      achieved HBM bytes and GB/s of every kernel family of a program: bytes per launch from a FETCH_SIZE
      run and a WRITE_SIZE run (scaled by the device copy in the same runs), average duration from a
      --kernel-trace --stats run of the same program
  python -m paper_2307_14123_amd.profiling mfma <pmc dir> <kernel_stats.csv> --command "<cmd>" --out <file.md>
      matrix-core and VALU counters per kernel family from one --pmc run of SQ_VALU_MFMA_BUSY_CYCLES,
      SQ_BUSY_CYCLES, SQ_INSTS_MFMA, SQ_INSTS_VALU, SQ_INSTS_VALU_MFMA_MOPS_F32, SQ_INSTS_VALU_MFMA_MOPS_BF16,
      SQ_LDS_BANK_CONFLICT, SQ_WAIT_INST_LDS and GRBM_GUI_ACTIVE, with durations from a --kernel-trace
      --stats run of the same program
  python -m paper_2307_14123_amd.profiling traffic <fetch dir> <write dir> --family "gemm_kernel<jet>"
      --source <csrc file> --command "<cmd>" --out <file.txt>
      HBM bytes per launch of one kernel family from a FETCH_SIZE run and a WRITE_SIZE run,
      each scaled by what the same counter reads for the plain device copy in the same run
      (bench.py --copy-calibration copies 256 MiB)

Only reads CSV files; nothing here touches the GPU.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os
import re

COPY_BYTES = 256 << 20


def family(kernel_name: str) -> str:
    """bench.py's family of a demangled kernel name ('qmc::gemm_kernel<1, 6, 2, 16, false>(...)')."""
    base = kernel_name.split("(")[0].replace("void ", "").strip()
    base = base.split("::")[-1] if base.startswith("qmc::") else base
    m = re.match(r"(\w+)<(.*)>$", base)
    if not m:
        return base
    name, targs = m.group(1), [t.strip() for t in m.group(2).split(",")]
    if name == "det_kernel" and len(targs) >= 3:
        return "det_kernel<" + ("inv" if targs[2] == "true" else "lu") + ">"
    if name == "gemm_kernel" and len(targs) >= 3:
        return "gemm_kernel<" + {"0": "val", "1": "edge", "2": "jet"}.get(targs[2], targs[2]) + ">"
    if name == "edge_mlp_kernel":
        return "edge_mlp_kernel<" + ("jet" if targs[0] == "1" else "val") + ">"
    if name in ("wgrad_kernel", "wgrad_f32_kernel"):
        return "wgrad_kernel"
    return name


def stats(path: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["# Kernel time summary", "", "Command (run from the repository root):", "", "    " + command, "",
           "| kernel | family | launches | total ms | average us | share |", "|---|---|---|---|---|---|"]
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    fam = collections.defaultdict(lambda: [0, 0.0])
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:30]:
        f = family(r["Name"])
        n, t = int(r["Calls"]), float(r["TotalDurationNs"])
        out.append(f"| `{r['Name'].split('(')[0][:70]}` | {f} | {n} | {t / 1e6:.3f} | {t / n / 1e3:.1f} | "
                   f"{100 * t / tot:.1f}% |")
    for r in rows:
        f = family(r["Name"])
        fam[f][0] += int(r["Calls"])
        fam[f][1] += float(r["TotalDurationNs"])
    out += ["", "| family | launches | total ms | average us |", "|---|---|---|---|"]
    for f, (n, t) in sorted(fam.items(), key=lambda kv: -kv[1][1])[:15]:
        out.append(f"| {f} | {n} | {t / 1e6:.3f} | {t / n / 1e3:.1f} |")
    return "\n".join(out) + "\n"


def _counter(d: str, counter: str):
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter:
                per[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return per


def traffic(fetch_dir: str, write_dir: str, fam: str, source: str, command: str) -> str:
    fetch, write = _counter(fetch_dir, "FETCH_SIZE"), _counter(write_dir, "WRITE_SIZE")

    def copy_kib(per):
        vals = [v for k, d in per.items() if "copyBuffer" in k for v in d.values()]
        if not vals:
            raise SystemExit("no device copy in the counter run (use bench.py --copy-calibration)")
        return max(vals)

    def fam_kib(per):
        vals = [v for k, d in per.items() if family(k) == fam for v in d.values()]
        if not vals:
            raise SystemExit(f"no launch of {fam} in the counter run")
        return sum(vals) / len(vals), len(vals)

    sf = COPY_BYTES / (copy_kib(fetch) * 1024.0)
    sw = COPY_BYTES / (copy_kib(write) * 1024.0)
    f_kib, nf = fam_kib(fetch)
    w_kib, nw = fam_kib(write)
    bytes_per_launch = f_kib * 1024.0 * sf + w_kib * 1024.0 * sw
    sha = hashlib.sha256(open(source, "rb").read()).hexdigest()
    lines = [
        f"# HBM traffic of {fam}",
        "command: " + command,
        f"kernel_family: {fam}",
        f"source: {os.path.relpath(source)}",
        f"source_sha256: {sha}",
        f"launches: {nf}",
        f"fetch_kib_per_launch_raw: {f_kib:.1f}",
        f"write_kib_per_launch_raw: {w_kib:.1f}",
        f"copy_fetch_scale: {sf:.4f}",
        f"copy_write_scale: {sw:.4f}",
        f"read_bytes_per_launch: {f_kib * 1024.0 * sf:.6g}",
        f"write_bytes_per_launch: {w_kib * 1024.0 * sw:.6g}",
        f"hbm_bytes_per_launch: {bytes_per_launch:.6g}",
    ]
    return "\n".join(lines) + "\n"


def hbm(fetch_dir: str, write_dir: str, stats_csv: str, command: str, top: int = 12) -> str:
    fetch, write = _counter(fetch_dir, "FETCH_SIZE"), _counter(write_dir, "WRITE_SIZE")

    def copy_kib(per):
        vals = [v for k, d in per.items() if "copyBuffer" in k for v in d.values()]
        if not vals:
            raise SystemExit("no device copy in the counter run")
        return max(vals)

    sf = COPY_BYTES / (copy_kib(fetch) * 1024.0)
    sw = COPY_BYTES / (copy_kib(write) * 1024.0)
    per_fam = collections.defaultdict(lambda: [0.0, 0.0, 0])  # read bytes, write bytes, launches
    for per, scale, slot in ((fetch, sf, 0), (write, sw, 1)):
        for k, d in per.items():
            if "copyBuffer" in k or "_peak_kernel" in k or not k.startswith(("qmc::", "void qmc::")):
                continue
            f = family(k)
            per_fam[f][slot] += sum(d.values()) * 1024.0 * scale
            if slot == 0:
                per_fam[f][2] += len(d)
    dur = collections.defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(stats_csv)):
        f = family(r["Name"])
        dur[f][0] += int(r["Calls"])
        dur[f][1] += float(r["TotalDurationNs"])
    out = ["# Achieved HBM traffic per kernel family", "", "Commands (run from the repository root):", "",
           "    " + command, "",
           f"Counter scaling from the device copy of {COPY_BYTES >> 20} MiB in the same runs: FETCH_SIZE x {sf:.4f}, "
           f"WRITE_SIZE x {sw:.4f}.", "",
           "| family | launches | MB read / launch | MB written / launch | average us | achieved GB/s |",
           "|---|---|---|---|---|---|"]
    rows = []
    for f, (rd, wr, n) in per_fam.items():
        if n == 0 or f not in dur or dur[f][0] == 0:
            continue
        avg_s = dur[f][1] / dur[f][0] * 1e-9
        rows.append((dur[f][1], f, n, rd / n, wr / n, avg_s))
    for _, f, n, rd, wr, avg_s in sorted(rows, reverse=True)[:top]:
        out.append(f"| {f} | {n} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | {avg_s * 1e6:.1f} | {(rd + wr) / avg_s / 1e9:.0f} |")
    return "\n".join(out) + "\n"


MFMA_COUNTERS = ("SQ_VALU_MFMA_BUSY_CYCLES", "SQ_BUSY_CYCLES", "SQ_INSTS_MFMA", "SQ_INSTS_VALU",
                 "SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_LDS_BANK_CONFLICT",
                 "SQ_WAIT_INST_LDS", "GRBM_GUI_ACTIVE")
SIMDS = 256 * 4  # MI355X: 256 compute units of 4 SIMDs
CLOCK_HZ = 2.4e9  # MI355X peak engine clock


def mfma(pmc_dir: str, stats_csv: str, command: str, top: int = 14) -> str:
    per = {c: _counter(pmc_dir, c) for c in MFMA_COUNTERS}
    fam = collections.defaultdict(lambda: collections.defaultdict(float))
    for c, d in per.items():
        for k, disp in d.items():
            if not k.startswith(("qmc::", "void qmc::")) or "_peak_kernel" in k:
                continue
            f = family(k)
            fam[f][c] += sum(disp.values())
            if c == "SQ_INSTS_MFMA":
                fam[f]["dispatches"] += len(disp)
    dur = collections.defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(stats_csv)):
        f = family(r["Name"])
        dur[f][0] += int(r["Calls"])
        dur[f][1] += float(r["TotalDurationNs"])
    out = ["# Matrix-core (MFMA) and VALU counters per kernel family", "", "Commands (run from the repository root):",
           "", "    " + command, "",
           "Columns, per dispatch of the family (sums over all dispatches of the counter run divided by their count; "
           "durations from the trace run):",
           f"- MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (average duration x {CLOCK_HZ / 1e9:.1f} GHz x {SIMDS} SIMDs): "
           "the share of SIMD-cycles in which the matrix core was busy (the counter is summed over the SIMDs);",
           "- MFMA TFLOP/s = SQ_INSTS_VALU_MFMA_MOPS_F32 x 512 flops / average duration: executed float32 MFMA work "
           "(padding rows included) per second; bf16 TFLOP/s the same from SQ_INSTS_VALU_MFMA_MOPS_BF16 (the edge "
           "filters' three-piece second layer: six bf16 products per float32 product);",
           "- VALU / MFMA = SQ_INSTS_VALU / SQ_INSTS_MFMA (SQ_INSTS_VALU counts the MFMA instructions too);",
           "- LDS bank-conflict cycles and LDS-issue waits (quad-cycles) per dispatch;",
           f"- GRBM / clk and SQ busy / clk: GRBM_GUI_ACTIVE and SQ_BUSY_CYCLES over average duration x "
           f"{CLOCK_HZ / 1e9:.1f} GHz, the number of counter instances summed (a check of the clock assumption).", "",
           "| family | dispatches | average us | MFMA busy | MFMA TFLOP/s (f32) | MFMA TFLOP/s (bf16) | "
           "MFMA insts / dispatch | VALU / MFMA | LDS bank-conflict cycles / dispatch | LDS wait / dispatch | "
           "GRBM / clk | SQ busy / clk |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    rows = []
    for f, v in fam.items():
        n = v.get("dispatches", 0)
        if n == 0 or f not in dur or dur[f][0] == 0:
            continue
        rows.append((dur[f][1], f, n, v))
    for _, f, n, v in sorted(rows, key=lambda t: t[0], reverse=True)[:top]:
        avg_s = dur[f][1] / dur[f][0] * 1e-9
        cyc = avg_s * CLOCK_HZ
        util = v["SQ_VALU_MFMA_BUSY_CYCLES"] / n / (cyc * SIMDS)
        tf = v["SQ_INSTS_VALU_MFMA_MOPS_F32"] * 512.0 / n / avg_s / 1e12
        tb = v["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512.0 / n / avg_s / 1e12
        ratio = v["SQ_INSTS_VALU"] / v["SQ_INSTS_MFMA"] if v["SQ_INSTS_MFMA"] > 0 else float("nan")
        out.append(f"| {f} | {n} | {avg_s * 1e6:.1f} | {100 * util:.1f}% | {tf:.1f} | {tb:.1f} | {v['SQ_INSTS_MFMA'] / n:.3g} | "
                   f"{ratio:.2f} | {v['SQ_LDS_BANK_CONFLICT'] / n:.3g} | {v['SQ_WAIT_INST_LDS'] / n:.3g} | "
                   f"{v['GRBM_GUI_ACTIVE'] / n / cyc:.2f} | {v['SQ_BUSY_CYCLES'] / n / cyc:.2f} |")
    out += ["", "Raw sums over the counter run:", "", "| family | " + " | ".join(MFMA_COUNTERS) + " |",
            "|---|" + "---|" * len(MFMA_COUNTERS)]
    for _, f, n, v in sorted(rows, key=lambda t: t[0], reverse=True)[:top]:
        out.append(f"| {f} | " + " | ".join(f"{v[c]:.4g}" for c in MFMA_COUNTERS) + " |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a1 = sub.add_parser("stats")
    a1.add_argument("csv")
    a1.add_argument("--command", required=True)
    a1.add_argument("--out", required=True)
    a2 = sub.add_parser("traffic")
    a2.add_argument("fetch_dir")
    a2.add_argument("write_dir")
    a2.add_argument("--family", required=True)
    a2.add_argument("--source", required=True)
    a2.add_argument("--command", required=True)
    a2.add_argument("--out", required=True)
    a3 = sub.add_parser("hbm")
    a3.add_argument("fetch_dir")
    a3.add_argument("write_dir")
    a3.add_argument("stats_csv")
    a3.add_argument("--command", required=True)
    a3.add_argument("--out", required=True)
    a4 = sub.add_parser("mfma")
    a4.add_argument("pmc_dir")
    a4.add_argument("stats_csv")
    a4.add_argument("--command", required=True)
    a4.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "mfma":
        text = mfma(args.pmc_dir, args.stats_csv, args.command)
    elif args.cmd == "hbm":
        text = hbm(args.fetch_dir, args.write_dir, args.stats_csv, args.command)
    elif args.cmd == "stats":
        text = stats(args.csv, args.command)
    else:
        text = traffic(args.fetch_dir, args.write_dir, args.family, args.source, args.command)
    with open(args.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
