"""Summaries of rocprofv3 output for the selected-inversion kernels.

Two jobs, both on the CSV files rocprofv3 writes with ``--output-format csv``:

``stats DIR``
    per-kernel dispatch statistics from ``*kernel_trace.csv``, split by the batch
    (grid y), printed as markdown tables.

``gaps DIR``
    launch gaps: the trace's dispatches split into phases wherever the device is idle
    for more than ``--idle-ms`` (bench.py ``--gap-phases`` separates its phases by
    sleeps); per phase the wall time from the first start to the last end, the sum of
    kernel durations, the time the device had a kernel running (union of intervals)
    and the idle fraction 1 - busy / wall, with the kernels that took the most time.

``traffic --fetch DIR --write DIR ...``
    HBM traffic per launch of one kernel from two ``--pmc`` passes (``FETCH_SIZE``,
    then ``WRITE_SIZE``, both in KiB per dispatch). Each counter is scaled by what it
    reads for a plain copy kernel of known size in the same process (bench.py
    ``--calibrate-copy`` runs one: it reads and writes ``--copy-bytes`` each), and the
    result is written as a JSON record together with the SHA-256 of the kernel's
    source, so that a reader can tell when the kernel has changed since the counters
    were taken.

    python -m paper_1707_08874_amd.profsum stats gpurun_out/ktrace
    python -m paper_1707_08874_amd.profsum traffic --fetch gpurun_out/pmc_fetch \\
        --write gpurun_out/pmc_write --kernel 'k_gemm<0, 2, 2>' --copy-kernel neg_kernel \\
        --copy-bytes 1073741824 --out paper_1707_08874_amd/traffic.json
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
GEMM_SOURCE = os.path.join(PKG, "csrc", "k_gemm.hip")


def source_digest(path: str = GEMM_SOURCE) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _rows(directory: str, suffix: str):
    files = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    for fn in files:
        with open(fn, newline="") as f:
            yield from csv.DictReader(f)


def short_name(name: str) -> str:
    """Kernel name without its parameter list ('void ns::k<1, 2>(args)' -> 'ns::k<1, 2>')."""
    n = name[5:] if name.startswith("void ") else name
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


def kernel_stats(directory: str):
    """{grid_y: {kernel: [durations in ms]}} from the kernel trace."""
    out = defaultdict(lambda: defaultdict(list))
    for r in _rows(directory, "kernel_trace.csv"):
        gy = int(r["Grid_Size_Y"]) // max(int(r["Workgroup_Size_Y"]), 1)
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
        out[gy][short_name(r["Kernel_Name"])].append(dur)
    return out


def stats_markdown(directory: str) -> str:
    lines = []
    for gy, ks in sorted(kernel_stats(directory).items(), key=lambda t: -t[0]):
        total = sum(sum(v) for v in ks.values())
        lines += [f"## Dispatches with grid y = {gy}", "",
                  "| kernel | calls | total ms | avg ms | min ms | max ms | share |",
                  "|---|---|---|---|---|---|---|"]
        for k, v in sorted(ks.items(), key=lambda t: -sum(t[1])):
            lines.append(f"| {k} | {len(v)} | {sum(v):.2f} | {sum(v) / len(v):.4f} | "
                         f"{min(v):.4f} | {max(v):.4f} | {100 * sum(v) / total:.1f}% |")
        lines.append("")
    return "\n".join(lines)


def gap_phases(directory: str, idle_ms: float = 50.0):
    """Phases of the kernel trace: lists of (start_ns, end_ns, kernel) split where no
    kernel runs for more than idle_ms."""
    ks = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]))
                for r in _rows(directory, "kernel_trace.csv"))
    phases, last_end = [], None
    for k in ks:
        if last_end is None or k[0] - last_end > idle_ms * 1e6:
            phases.append([])
        phases[-1].append(k)
        last_end = k[1] if last_end is None else max(last_end, k[1])
    return phases


def gaps_markdown(directory: str, idle_ms: float = 50.0, top: int = 8) -> str:
    lines = ["| phase | dispatches | wall ms | kernel sum ms | busy ms | idle fraction |",
             "|---|---|---|---|---|---|"]
    details = []
    for i, ph in enumerate(gap_phases(directory, idle_ms)):
        t0, t1 = ph[0][0], max(e for _, e, _ in ph)
        busy, cs, ce = 0, None, None
        for b, e, _ in ph:
            if ce is None or b > ce:
                if ce is not None:
                    busy += ce - cs
                cs, ce = b, e
            else:
                ce = max(ce, e)
        busy += ce - cs
        ksum = sum(e - b for b, e, _ in ph)
        lines.append(f"| {i} | {len(ph)} | {(t1 - t0) * 1e-6:.2f} | {ksum * 1e-6:.2f} | {busy * 1e-6:.2f} | "
                     f"{1 - busy / max(t1 - t0, 1):.4f} |")
        agg = defaultdict(lambda: [0, 0])
        for b, e, n in ph:
            agg[n][0] += 1
            agg[n][1] += e - b
        details += ["", f"Phase {i}: kernels by time", "", "| kernel | dispatches | ms | share |", "|---|---|---|---|"]
        for n, (c, t) in sorted(agg.items(), key=lambda x: -x[1][1])[:top]:
            details.append(f"| {n} | {c} | {t * 1e-6:.2f} | {100 * t / max(ksum, 1):.1f}% |")
    return "\n".join(lines + details)


def counter_per_dispatch(directory: str, counter: str, pattern: str):
    """Values of one counter for every dispatch whose kernel name matches the pattern."""
    rx = re.compile(pattern)
    vals = defaultdict(float)
    for r in _rows(directory, "counter_collection.csv"):
        if r["Counter_Name"] != counter or not rx.search(r["Kernel_Name"]):
            continue
        vals[int(r["Dispatch_Id"])] += float(r["Counter_Value"])
    if not vals:
        raise ValueError(f"no {counter} values for kernels matching {pattern!r} in {directory}")
    return [vals[k] for k in sorted(vals)]


def traffic_record(fetch_dir, write_dir, kernel, copy_kernel, copy_bytes):
    kf = counter_per_dispatch(fetch_dir, "FETCH_SIZE", re.escape(kernel))
    kw = counter_per_dispatch(write_dir, "WRITE_SIZE", re.escape(kernel))
    cf = counter_per_dispatch(fetch_dir, "FETCH_SIZE", copy_kernel)
    cw = counter_per_dispatch(write_dir, "WRITE_SIZE", copy_kernel)
    # KiB -> bytes, then the copy kernel's reading of its known size fixes the scale
    f_fetch = copy_bytes / (1024.0 * sum(cf) / len(cf))
    f_write = copy_bytes / (1024.0 * sum(cw) / len(cw))
    fetch = 1024.0 * f_fetch * sum(kf) / len(kf)
    write = 1024.0 * f_write * sum(kw) / len(kw)
    return {
        "kernel": kernel,
        "source_sha256": source_digest(),
        "dispatches": len(kf),
        "fetch_bytes_per_launch": fetch,
        "write_bytes_per_launch": write,
        "bytes_per_launch": fetch + write,
        "copy_kernel": copy_kernel,
        "copy_bytes": copy_bytes,
        "copy_fetch_factor": f_fetch,
        "copy_write_factor": f_write,
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    gp = sub.add_parser("gaps")
    gp.add_argument("dir")
    gp.add_argument("--idle-ms", type=float, default=50.0)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True, help="substring of the demangled kernel name")
    t.add_argument("--copy-kernel", required=True, help="regex for the calibration copy kernel")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--workload", type=json.loads, default=None,
                   help="JSON object naming the workload the counters were taken on")
    t.add_argument("--command", default="", help="the profiled command, for the record")
    t.add_argument("--bench-log", default=None,
                   help="output of the profiled bench run: its JSON line supplies the algorithmic "
                        "bytes per launch, which identify the launch set the counters belong to")
    t.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_markdown(a.dir))
        return 0
    if a.cmd == "gaps":
        print(gaps_markdown(a.dir, a.idle_ms))
        return 0
    rec = traffic_record(a.fetch, a.write, a.kernel, a.copy_kernel, a.copy_bytes)
    rec["workload"] = a.workload
    rec["command"] = a.command
    if a.bench_log:
        line = [ln for ln in open(a.bench_log) if ln.lstrip().startswith("{")][-1]
        roof = json.loads(line)["roofline"]
        rec["alg_bytes_per_launch"] = roof["alg_bytes_per_launch"]
        rec["traffic_over_alg"] = rec["bytes_per_launch"] / roof["alg_bytes_per_launch"]
    text = json.dumps(rec, indent=1, sort_keys=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
