#!/usr/bin/env python3
"""Collect rocprofv3 hardware counters for one kernel and write the summary
kept under profiles/.

    python3 profile_counters.py --kernel 'forward_kernel<2048' \\
        --out profiles/forward_L2048_2e21x85_counters.md --title '...' \\
        -- python3 bench.py --steps 3 --warmup 1 --no-extras --no-cpu-baseline --L 2048

Every counter pass is its own rocprofv3 run of the command (rocprofv3 does not
split counters over passes), started as a child process under a hard time
limit; this script itself never touches the GPU.  The selected kernel's
dispatches must all have the same grid and workgroup size (a summary is one
kernel at one size), and the mean over them is reported.  HBM traffic is
FETCH_SIZE and WRITE_SIZE scaled by what the same counters read for a plain
device copy of known size (the command is expected to run one first:
bench.py --copy-calibration BYTES).  The summary records the sha256 of the
library sources it was taken from; bench.py uses its traffic and VALU figures
only while that hash matches.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import shlex
import subprocess
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# one pass per run: at most 8 SQ, 4 TCC (FETCH_SIZE takes 3, WRITE_SIZE 2)
# and 2 GRBM counters each
PASSES = [
    ["FETCH_SIZE"],
    ["WRITE_SIZE"],
    ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU"],
    ["SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_ACTIVE_INST_VALU", "SQ_LDS_BANK_CONFLICT"],
    ["GRBM_GUI_ACTIVE", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_ACTIVE_INST_LDS"],
]
COPY_KERNEL = "__amd_rocclr_copyBuffer"
XCDS = 8
SIMDS = 256 * 4


def run_pass(counters, cmd, outdir, limit):
    os.makedirs(outdir, exist_ok=True)
    full = ["timeout", "-s", "KILL", str(limit), "rocprofv3", "--pmc", *counters, "-f", "csv",
            "-d", outdir, "-o", "p", "--", *cmd]
    print("# " + " ".join(shlex.quote(c) for c in full), flush=True)
    with open(os.path.join(outdir, "run.log"), "w") as log:
        rc = subprocess.run(full, stdout=log, stderr=subprocess.STDOUT).returncode
    files = glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True)
    if rc != 0 and not files:
        raise SystemExit(f"rocprofv3 pass {counters} failed with status {rc} (see {outdir})")
    rows = []
    for f in files:
        rows.extend(csv.DictReader(open(f)))
    return rows


def dispatches(rows, match):
    """{dispatch id: (kernel name, grid, workgroup, {counter: value})} of the
    kernels whose name contains `match`."""
    out = {}
    for r in rows:
        if match not in r["Kernel_Name"]:
            continue
        d = out.setdefault(int(r["Dispatch_Id"]),
                           (r["Kernel_Name"], int(r["Grid_Size"]), int(r["Workgroup_Size"]),
                            int(r["LDS_Block_Size"]), {}))
        d[4][r["Counter_Name"]] = d[4].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def trace(args, cmd) -> int:
    """--trace: one rocprofv3 --kernel-trace --stats run; the summary lists the
    calls and mean / min / max duration of every kernel matching --kernel
    (a comma-separated list of name substrings)."""
    from bench import kernel_sources_hash

    outdir = args.workdir
    os.makedirs(outdir, exist_ok=True)
    full = ["timeout", "-s", "KILL", str(args.limit), "rocprofv3", "--kernel-trace", "--stats",
            "-f", "csv", "-d", outdir, "-o", "t", "--", *cmd]
    print("# " + " ".join(shlex.quote(c) for c in full), flush=True)
    with open(os.path.join(outdir, "run.log"), "w") as log:
        rc = subprocess.run(full, stdout=log, stderr=subprocess.STDOUT).returncode
    files = glob.glob(os.path.join(outdir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit(f"rocprofv3 trace failed with status {rc} (see {outdir})")
    rows = list(csv.DictReader(open(files[0])))
    pats = [p for p in args.kernel.split(",") if p]
    cmdline = "python3 profile_counters.py " + " ".join(shlex.quote(a) for a in sys.argv[1:])
    lines = [f"# {args.title}", "", "Made by (from the repository root, TMPDIR=/tmp):", "",
             f"    {cmdline}", "", "which runs:", "",
             "    rocprofv3 --kernel-trace --stats -f csv -d <out> -o t -- " +
             " ".join(shlex.quote(c) for c in cmd), "",
             "| kernel | calls | mean us | min us | max us |", "|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        if pats and not any(p in r["Name"] for p in pats):
            continue
        lines.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
    if args.note:
        lines += ["", args.note]
    files_h = args.sources.split() or None
    lines += ["", f"kernel_sources: {' '.join(sorted(files_h)) if files_h else ''}",
              f"kernel_sources_hash: {kernel_sources_hash(files_h)}", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print(f"# wrote {args.out}", flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--kernel", required=True, help="substring of the kernel's name")
    ap.add_argument("--trace", action="store_true",
                    help="a kernel trace with per-kernel duration statistics instead of counters")
    ap.add_argument("--out", required=True, help="summary file (Markdown)")
    ap.add_argument("--title", required=True)
    ap.add_argument("--note", default="", help="paragraph appended to the summary")
    ap.add_argument("--workdir", default="gpurun_out/counters")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30,
                    help="bytes the command's calibration copy reads and writes")
    ap.add_argument("--limit", type=int, default=150, help="seconds per pass")
    ap.add_argument("--algorithmic-bytes", type=float, default=0.0,
                    help="algorithmic HBM bytes per launch, for the comparison line")
    ap.add_argument("--grid-size", type=int, default=0,
                    help="only dispatches of this grid size (total lanes)")
    ap.add_argument("--largest", action="store_true",
                    help="only the dispatches of the largest grid size among the matches")
    ap.add_argument("--sources", default="",
                    help="the csrc/ files the kernel is built from (space-separated; "
                         "default: all of csrc/), hashed into the summary")
    ap.add_argument("cmd", nargs=argparse.REMAINDER)
    args = ap.parse_args()
    cmd = args.cmd[1:] if args.cmd[:1] == ["--"] else args.cmd
    if not cmd:
        ap.error("no command after --")
    if args.trace:
        return trace(args, cmd)
    from bench import kernel_sources_hash

    values, names, shapes, calib, commands = {}, set(), set(), {}, []
    for i, counters in enumerate(PASSES):
        rows = run_pass(counters, cmd, os.path.join(args.workdir, f"pass{i}"), args.limit)
        commands.append("rocprofv3 --pmc " + " ".join(counters) + " -f csv -d <out> -o p -- " +
                        " ".join(shlex.quote(c) for c in cmd))
        sel = dispatches(rows, args.kernel)
        if args.grid_size:
            sel = {k: v for k, v in sel.items() if v[1] == args.grid_size}
        if args.largest and sel:
            top = max(v[1] for v in sel.values())
            sel = {k: v for k, v in sel.items() if v[1] == top}
        if not sel:
            raise SystemExit(f"no dispatch of a kernel matching {args.kernel!r} in pass {counters}")
        for name, grid, wg, lds, cv in sel.values():
            names.add(name)
            shapes.add((grid, wg, lds))
            for c, v in cv.items():
                values.setdefault(c, []).append(v)
        for _, _, _, _, cv in dispatches(rows, COPY_KERNEL).values():
            for c in ("FETCH_SIZE", "WRITE_SIZE"):
                if c in cv:
                    calib[c] = max(calib.get(c, 0.0), cv[c])
    if len(names) != 1 or len(shapes) != 1:
        raise SystemExit(f"the match covers several kernels or sizes: {sorted(names)} {shapes}")
    name = names.pop()
    grid, wg, lds = shapes.pop()
    mean = {c: sum(v) / len(v) for c, v in values.items()}
    ndisp = min(len(v) for v in values.values())
    kib = args.copy_bytes / 1024
    fs = kib / calib["FETCH_SIZE"] if calib.get("FETCH_SIZE") else 1.0
    ws = kib / calib["WRITE_SIZE"] if calib.get("WRITE_SIZE") else 1.0
    fetch = mean.get("FETCH_SIZE", 0.0) * fs * 1024
    write = mean.get("WRITE_SIZE", 0.0) * ws * 1024
    cycles = mean.get("GRBM_GUI_ACTIVE", 0.0) / XCDS
    valu = mean.get("SQ_INSTS_VALU", 0.0)
    issue = valu * 4 / (cycles * SIMDS) if cycles else 0.0

    cmdline = "python3 profile_counters.py " + " ".join(shlex.quote(a) for a in sys.argv[1:])
    lines = [f"# {args.title}", "",
             f"Kernel: `{name}`, mean over {ndisp} dispatches of one size.",
             f"Launch: grid {grid // wg} workgroups x {wg} lanes, LDS {lds} B per workgroup.",
             "Sources: `kernel_sources_hash` below (sha256 over the csrc/ files named in "
             "`kernel_sources`, or all of paper_1804_05335_amd/csrc/, first 16 hex).", "",
             "Made by (from the repository root, TMPDIR=/tmp):", "", f"    {cmdline}", "",
             "which makes one rocprofv3 run per counter pass:", ""]
    lines += [f"    {c}" for c in commands]
    lines += ["", f"## Calibration: plain device copy of {args.copy_bytes} B (`{COPY_KERNEL}`)", ""]
    if calib:
        lines.append(f"FETCH_SIZE = {calib.get('FETCH_SIZE', 0):.0f} KiB (scale x{fs:.3f}); "
                     f"WRITE_SIZE = {calib.get('WRITE_SIZE', 0):.0f} KiB (scale x{ws:.3f}).")
    else:
        lines.append("No calibration copy found: FETCH_SIZE and WRITE_SIZE taken unscaled.")
    lines += ["", "## Counters (mean per dispatch)", "", "| counter | value |", "|---|---|"]
    for c in sorted(mean):
        lines.append(f"| {c} | {mean[c]:.5g} |")
    lines += ["",
              f"GRBM_GUI_ACTIVE / {XCDS} XCDs = {cycles:.4g} cycles per dispatch.",
              f"VALU issue: SQ_INSTS_VALU x 4 cycles / (cycles x {SIMDS} SIMDs) = "
              f"{100 * issue:.1f} % of the VALU issue slots."]
    if "SQ_INSTS_LDS" in mean and "SQ_LDS_BANK_CONFLICT" in mean:
        lines.append(f"LDS: SQ_LDS_BANK_CONFLICT = {mean['SQ_LDS_BANK_CONFLICT']:.4g} cycles for "
                     f"SQ_INSTS_LDS = {mean['SQ_INSTS_LDS']:.4g} instructions "
                     f"(ratio {mean['SQ_LDS_BANK_CONFLICT'] / max(mean['SQ_INSTS_LDS'], 1):.3f}).")
    alg = (f" (algorithmic {args.algorithmic_bytes / 1e6:.1f} MB)"
           if args.algorithmic_bytes else "")
    lines.append(f"HBM traffic per launch: {fetch / 1e6:.1f} MB read + {write / 1e6:.1f} MB "
                 f"written = {(fetch + write) / 1e6:.1f} MB{alg}.")
    if args.note:
        lines += ["", args.note]
    files = args.sources.split() or None
    lines += ["", f"kernel_sources: {' '.join(sorted(files)) if files else ''}",
              f"kernel_sources_hash: {kernel_sources_hash(files)}",
              f"fetch_bytes_per_launch: {fetch:.0f}",
              f"write_bytes_per_launch: {write:.0f}",
              f"valu_insts_per_launch: {valu:.0f}",
              f"cycles_per_launch: {cycles:.0f}", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print(f"# wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
