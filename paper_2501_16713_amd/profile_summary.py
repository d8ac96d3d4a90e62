"""Profile bench.py with rocprofv3 and summarise it per operator stage.

Three runs of the same bench command, each in a process of its own:

  1. --kernel-trace --stats   per-kernel durations
  2. --pmc FETCH_SIZE         HBM bytes read per dispatch (KiB)
  3. --pmc WRITE_SIZE         HBM bytes written per dispatch (KiB)

The bench is run with --calib-copy-mb, so each process also launches one
plain elementwise kernel (a negation) that reads and writes a known number
of bytes; both counters are scaled by what they read for it.

    python3 -m paper_2501_16713_amd.profile_summary --out out/normal_op_batched_160_fp32 \\
        --raw out/prof_raw -- --steps 3 --warmup 1 --cg-iters 0 --no-cpu-baseline --forms "" \\
        --no-rows --no-tune --kblock 2 --ktile 4 --chunk 1024 --batch 6 --graph 0

writes OUT.md (the table, with the commands) and OUT.json (read by bench.py,
which reports the traffic of its dominant stage only while the kernel
sources still hash to the value recorded there).  With --parse-only the runs
are skipped and the raw directories are only summarised.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import shlex
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def csrc_hash() -> str:
    """sha256 over the kernel sources (file names and contents)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stage_of(kernel: str) -> str:
    """Map a demangled kernel name to the library's timing tag."""
    if "neg_kernel" in kernel:
        return "calibration_copy"
    if "rocclr_copyBuffer" in kernel:
        return "runtime_copy (plan-time uploads)"
    if "kspread_reduce" in kernel:
        return "kspread_reduce"
    if "kspread_kernel" in kernel or "kspread_reg_kernel" in kernel:
        return "kspread"
    if "kgather_kernel" in kernel:
        return "kgather"
    if "visit_permute" in kernel:
        return "visit_permute"
    for tag in ("warp_spread", "warp_gather", "warp_grad"):
        if tag + "_kernel" in kernel:
            return tag
    if "fft2_kernel" in kernel:
        if "Ld2Image" in kernel:
            return "fft_upsample_passes"
        if "Ld2CoilExpand" in kernel:
            return "fft_coil_fwd_last"
        if "St2CoilReduce" in kernel:
            return "fft_coil_adj_last"
        if "St2Masked" in kernel:
            return "fft_coil_fwd_ax0"
        if "Ld2Masked" in kernel or "Ld2Tiles" in kernel:
            return "fft_coil_adj_ax0"
        m = re.search(r"fft2_kernel<\d+, \d+, (-?\d+)", kernel)
        return "fft_coil_fwd_ax1" if m and m.group(1).startswith("-") else "fft_coil_adj_ax1"
    if "fft_pass_kernel" in kernel:
        return "fft_upsample_passes"
    m = re.search(r"isg::(\w+)_kernel", kernel)
    return m.group(1) if m else "other: " + kernel.split("(")[0][:60]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def trace_stats(d: str) -> dict:
    """stage -> [dispatches, average ms] from the kernel trace"""
    acc = collections.defaultdict(list)
    with open(_find(d, "kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            acc[stage_of(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
    return {k: [len(v), sum(v) / len(v)] for k, v in acc.items()}


def kernel_stats(d: str, top: int = 12) -> list:
    """the --stats table: (kernel, calls, average ms, percent), largest first"""
    rows = []
    try:
        path = _find(d, "kernel_stats.csv")
    except FileNotFoundError:
        return rows
    with open(path) as f:
        for r in csv.DictReader(f):
            try:
                rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) * 1e-6, float(r["Percentage"])))
            except (KeyError, ValueError):
                continue
    rows.sort(key=lambda r: -r[3])
    return rows[:top]


def counter_per_dispatch(d: str, counter: str) -> dict:
    """stage -> average of the counter per dispatch (KiB for FETCH/WRITE_SIZE)"""
    vals = collections.defaultdict(lambda: collections.defaultdict(float))
    with open(_find(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                vals[stage_of(r["Kernel_Name"])][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {k: sum(v.values()) / len(v) for k, v in vals.items()}


def run_profiles(raw: str, bench_args: list, copy_mb: int, limit: int) -> list:
    """Run the three rocprofv3 passes; returns the command lines."""
    bench = ["python3", "bench.py"] + bench_args + ["--calib-copy-mb", str(copy_mb)]
    passes = [("trace", ["--kernel-trace", "--stats"]), ("fetch", ["--pmc", "FETCH_SIZE"]),
              ("write", ["--pmc", "WRITE_SIZE"])]
    env = dict(os.environ, TMPDIR="/tmp")
    cmds = []
    for name, opts in passes:
        out = os.path.join(raw, name)
        os.makedirs(out, exist_ok=True)
        cmd = (["timeout", "-s", "KILL", str(limit), "rocprofv3"] + opts +
               ["--output-format", "csv", "-d", out, "-o", name, "--"] + bench)
        line = " ".join(shlex.quote(c) for c in cmd)
        cmds.append(line)
        print(f"[profile] pass {name}: {line}", flush=True)
        with open(os.path.join(raw, f"{name}.log"), "w") as log:
            rc = subprocess.call(cmd, cwd=ROOT, env=env, stdout=log, stderr=subprocess.STDOUT)
        with open(os.path.join(raw, f"{name}.log")) as log:
            text = log.read()
        finished = '"metric"' in text
        print(f"[profile] pass {name}: exit {rc}, bench line printed: {finished}", flush=True)
        # rocprofv3 may itself end with SIGSEGV after the program has finished
        # and its results are complete; anything else stops the profiling
        if rc != 0 and not (rc in (139, -11) and finished):
            sys.exit(rc if rc > 0 else 1)
    return cmds


def summarise(raw: str, copy_mb: int, workload: str, commands: list, out: str) -> dict:
    times = trace_stats(os.path.join(raw, "trace"))
    kstats = kernel_stats(os.path.join(raw, "trace"))
    fetch = counter_per_dispatch(os.path.join(raw, "fetch"), "FETCH_SIZE")
    write = counter_per_dispatch(os.path.join(raw, "write"), "WRITE_SIZE")
    copy_bytes = copy_mb << 20
    kf = copy_bytes / (fetch["calibration_copy"] * 1024.0)  # bytes per KiB counted
    kw = copy_bytes / (write["calibration_copy"] * 1024.0)
    stages = {}
    for st, (n, ms) in sorted(times.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        if st == "calibration_copy":
            continue
        fb = fetch.get(st, 0.0) * 1024.0 * kf
        wb = write.get(st, 0.0) * 1024.0 * kw
        stages[st] = {"dispatches": n, "avg_ms": round(ms, 5), "fetch_bytes": int(fb), "write_bytes": int(wb),
                      "traffic_bytes": int(fb + wb),
                      "measured_GBps": round((fb + wb) / (ms * 1e-3) / 1e9, 1) if ms > 0 else None}
    rec = {"workload": workload, "csrc_hash": csrc_hash(), "commands": commands, "copy_mb": copy_mb,
           "calibration": {"fetch_bytes_per_KiB": kf, "write_bytes_per_KiB": kw}, "stages": stages}
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"# rocprofv3: normal operator, workload {workload}", "",
             "Commands (from the repository root, each a process of its own):", ""]
    lines += [f"    {c}" for c in commands]
    lines += ["", f"Kernel sources hash `{rec['csrc_hash']}`.  HBM counters are scaled by a plain elementwise "
              f"kernel that reads and writes {copy_mb} MiB in the same process: FETCH_SIZE x {kf:.4f}, "
              f"WRITE_SIZE x {kw:.4f} bytes per KiB counted.", "",
              "## Per stage (kernel trace durations; HBM bytes per dispatch from the counters)", "",
              "| stage | dispatches | avg ms | fetch MB | write MB | HBM GB/s |", "|---|---|---|---|---|---|"]
    for st, v in stages.items():
        lines.append(f"| {st} | {v['dispatches']} | {v['avg_ms']:.4f} | {v['fetch_bytes'] / 1e6:.1f} | "
                     f"{v['write_bytes'] / 1e6:.1f} | {v['measured_GBps']} |")
    lines += ["", "## rocprofv3 --stats (largest total time first)", "",
              "| kernel | calls | avg ms | % time |", "|---|---|---|---|"]
    for name, calls, ms, pct in kstats:
        short = name.split("(")[0].replace("|", "/")
        lines.append(f"| `{short[:150]}` | {calls} | {ms:.4f} | {pct:.2f} |")
    with open(out + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines), flush=True)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True, help="summary path without extension")
    ap.add_argument("--raw", required=True, help="directory for the raw rocprofv3 output")
    ap.add_argument("--copy-mb", type=int, default=2048)
    ap.add_argument("--workload", default="batched_160")
    ap.add_argument("--limit", type=int, default=240, help="seconds allowed per rocprofv3 run")
    ap.add_argument("--parse-only", action="store_true")
    ap.add_argument("bench_args", nargs=argparse.REMAINDER, help="-- then the bench.py arguments")
    args = ap.parse_args()
    bench_args = [a for a in args.bench_args if a != "--"]
    if "--workload" not in bench_args:
        bench_args += ["--workload", args.workload]
    if args.parse_only:
        with open(os.path.join(args.raw, "commands.json")) as f:
            commands = json.load(f)
    else:
        top = "python3 -m paper_2501_16713_amd.profile_summary " + " ".join(shlex.quote(a) for a in sys.argv[1:])
        commands = [top, "which ran:"] + run_profiles(args.raw, bench_args, args.copy_mb, args.limit)
        with open(os.path.join(args.raw, "commands.json"), "w") as f:
            json.dump(commands, f)
    summarise(args.raw, args.copy_mb, args.workload, commands, args.out)


if __name__ == "__main__":
    main()
