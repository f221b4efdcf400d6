"""Summaries of rocprofv3 runs of bench.py for the stencil kernels.

Two kinds, each written as a short markdown file:

  trace     per-kernel dispatch statistics from a `--kernel-trace --stats`
            run, plus the average duration of the launches inside the timed
            region (the last launches of each kernel, as many as the
            benchmark's own JSON line reports), next to the benchmark's HIP
            event average for the same launches;
  counters  HBM bytes per launch from one FETCH_SIZE and one WRITE_SIZE run,
            each scaled by what the same counter reads for the benchmark's
            plain device copy of known size (`--copy-probe-mb`);
  stats     per-kernel dispatch statistics of any run (the preconditioner
            network's kernels, the TV kernel), with the run's JSON line.

The counter summary carries the hash of the stencil kernel sources, so the
benchmark reports measured traffic only for the kernels that were profiled.

    python -m paper_2506_20513_amd.rocprof_summary trace --run-dir D --bench-json J \
        --command "..." --out profiles/X.md
    python -m paper_2506_20513_amd.rocprof_summary counters --fetch-dir D1 --fetch-json J1 \
        --write-dir D2 --write-json J2 --copy-mb 1024 --command-fetch "..." \
        --command-write "..." --out profiles/Y.md
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
# the kernels, and the host code that picks their launch decomposition
KERNEL_SOURCES = ("csrc/fwi_stream.hip", "csrc/fwi_internal.h", "csrc/fwi_host.cpp")
STENCIL = ("k_fwd_sweep", "k_fwd_reforward", "k_adj")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def _code_only(text: str) -> str:
    """Source text without comments and with runs of white space collapsed,
    so that a change of comments alone keeps the hash."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def short_name(name: str) -> str | None:
    """The benchmark's name for a kernel of a trace: the single-problem
    forward kernel k_fwd<K, TAIL, LEV> is k_fwd_sweep for LEV = 0 (only the
    final state written) and k_fwd_reforward for LEV = 1 (every level's Ez
    written); other kernels keep their own name."""
    m = re.search(r"::(k_\w+)<([^>]*)>", name)
    if not m:
        return None
    if m.group(1) == "k_fwd":
        lev = m.group(2).split(",")[-1].strip()
        return {"0": "k_fwd_sweep", "1": "k_fwd_reforward"}.get(lev, "k_fwd")
    return m.group(1)


def _csv(run_dir: str, suffix: str):
    files = sorted(glob.glob(os.path.join(run_dir, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {run_dir}")
    with open(files[0], newline="") as f:
        return list(csv.DictReader(f))


def _bench_line(path: str) -> dict:
    """The benchmark's JSON line (the last line of `path` that parses)."""
    with open(path) as f:
        lines = [ln for ln in f.read().splitlines() if ln.strip().startswith("{")]
    if not lines:
        raise SystemExit(f"no JSON line in {path}")
    return json.loads(lines[-1])


def _timed_launches(bench: dict, kernel: str) -> int:
    return int(bench["kernels"][kernel]["launches_per_step"]) * int(bench["steps"])


def trace_summary(a) -> str:
    stats = _csv(a.run_dir, "kernel_stats.csv")
    trace = _csv(a.run_dir, "kernel_trace.csv")
    bench = _bench_line(a.bench_json)
    out = [f"# rocprofv3 kernel trace: stencil kernels, {bench['config']['workload']}", "",
           "Command (from the repository root):", "", "```", a.command, "```", "",
           f"Kernel sources hash: `{kernel_source_hash()}`", "",
           "## All dispatches (rocprofv3 --stats)", "",
           "| kernel | calls | avg us | min us | max us | total s | % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:12]:
        out.append(f"| `{r['Name'][:70]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e9:.3f} | {float(r['Percentage']):.2f} |")
    out += ["", "## Timed region: last launches of each stencil kernel", "",
            "| kernel | launches | rocprofv3 avg ms | bench HIP-event avg ms | ratio |",
            "|---|---:|---:|---:|---:|"]
    for k in STENCIL:
        if k not in bench["kernels"]:
            continue
        n = _timed_launches(bench, k)
        d = [(int(r["Dispatch_Id"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
             for r in trace if short_name(r["Kernel_Name"]) == k]
        d.sort()
        sel = [ms for _, ms in d[-n:]]
        avg = sum(sel) / len(sel)
        hip = bench["kernels"][k]["avg_ms"]
        out.append(f"| {k} | {len(sel)} | {avg:.4f} | {hip:.4f} | {avg / hip:.4f} |")
    out += ["", f"Benchmark line of this run: value {bench['value']} {bench['unit']}, "
                f"{bench['ms_per_step']} ms per step.", ""]
    return "\n".join(out)


def _counter(run_dir: str, bench: dict, copy_bytes: float):
    rows = _csv(run_dir, "counter_collection.csv")
    name = rows[0]["Counter_Name"]
    per = {}
    copies = []
    for r in rows:
        k = short_name(r["Kernel_Name"])
        v = float(r["Counter_Value"]) * 1024.0      # KiB -> bytes
        if k in STENCIL:
            per.setdefault(k, []).append((int(r["Dispatch_Id"]), v))
        elif r["Kernel_Name"].startswith(COPY_KERNEL):
            copies.append((int(r["Grid_Size"]), v))
    if not copies:
        raise SystemExit(f"{run_dir}: no {COPY_KERNEL} dispatch for the calibration")
    probe = max(copies)[1]                          # the large copy of the probe
    factor = copy_bytes / probe
    res = {}
    for k, d in per.items():
        d.sort()
        n = _timed_launches(bench, k)
        sel = [v for _, v in d[-n:]]
        res[k] = {"launches": len(sel), "raw": sum(sel) / len(sel), "factor": factor}
    return name, probe, factor, res


def counters_summary(a) -> str:
    copy_bytes = a.copy_mb * float(1 << 20)
    bf = _bench_line(a.fetch_json)
    bw = _bench_line(a.write_json)
    fn, fprobe, ff, fres = _counter(a.fetch_dir, bf, copy_bytes)
    wn, wprobe, wf, wres = _counter(a.write_dir, bw, copy_bytes)
    out = [f"# rocprofv3 HBM counters: stencil kernels, {bf['config']['workload']}", "",
           "Commands (from the repository root):", "", "```", a.command_fetch,
           a.command_write, "```", "",
           f"Kernel sources hash: `{kernel_source_hash()}`", "",
           "## Calibration: plain device copy of "
           f"{a.copy_mb} MiB (reads and writes {copy_bytes / 1e9:.3f} GB)", "",
           "| counter | reads for the copy | scale factor |", "|---|---:|---:|",
           f"| {fn} | {fprobe / 1e9:.4f} GB | {ff:.4f} |",
           f"| {wn} | {wprobe / 1e9:.4f} GB | {wf:.4f} |", "",
           "## Per launch (timed gradient only)", "",
           "| kernel | launches | fetch GB | write GB | traffic GB | algorithmic GB | traffic / algorithmic |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    machine = {"kernel_sources": kernel_source_hash(), "workload": bf["config"]["workload"],
               "grid": bf["config"]["grid"], "shots": bf["config"]["shots"], "kernels": {}}
    for k in STENCIL:
        if k not in fres or k not in wres:
            continue
        fb = fres[k]["raw"] * ff
        wb = wres[k]["raw"] * wf
        alg = bf["kernels"][k]["bytes_per_launch"]
        out.append(f"| {k} | {fres[k]['launches']} | {fb / 1e9:.4f} | {wb / 1e9:.4f} | "
                   f"{(fb + wb) / 1e9:.4f} | {alg / 1e9:.4f} | {(fb + wb) / alg:.4f} |")
        machine["kernels"][k] = {"fetch_bytes": fb, "write_bytes": wb,
                                 "traffic_bytes": fb + wb, "algorithmic_bytes": alg}
    out += ["", "Machine-readable (read by bench.py):", "", "```json",
            json.dumps(machine), "```", ""]
    return "\n".join(out)


def read_traffic(path: str, kernel: str, grid, shots: int):
    """Measured HBM bytes per launch of `kernel` from a counter summary, or
    None when the summary is missing, covers another workload, or was taken
    on other kernel sources."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        text = f.read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_sources") != kernel_source_hash():
        return None
    if list(d.get("grid", [])) != list(grid) or d.get("shots") != shots:
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else float(k["traffic_bytes"])


def stats_summary(a) -> str:
    """Per-kernel dispatch statistics of any run, with the program's own
    JSON result line (for kernels other than the stencils)."""
    stats = _csv(a.run_dir, "kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in stats)
    src = hashlib.sha256()
    for rel in a.sources.split(","):
        with open(os.path.join(HERE, rel), "rb") as f:
            src.update(f.read())
    out = [f"# rocprofv3 kernel statistics: {a.title}", "",
           "Command (from the repository root):", "", "```", a.command, "```", "",
           f"Kernel sources ({a.sources}) hash: `{src.hexdigest()[:16]}`", "",
           "| kernel | calls | avg us | min us | max us | total ms | % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:a.top]:
        name = r["Name"].replace("(anonymous namespace)::", "").replace("|", "/")[:80]
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{100.0 * float(r['TotalDurationNs']) / tot:.1f} |")
    if a.result_json:
        out += ["", "Result line of the profiled run:", "", "```json",
                json.dumps(_bench_line(a.result_json)), "```"]
    out.append("")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="kind", required=True)
    k = sub.add_parser("stats")
    k.add_argument("--run-dir", required=True)
    k.add_argument("--title", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--sources", required=True,
                   help="comma-separated kernel sources relative to the package")
    k.add_argument("--result-json", default=None)
    k.add_argument("--top", type=int, default=16)
    k.add_argument("--out", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--run-dir", required=True)
    t.add_argument("--bench-json", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    for x in ("fetch-dir", "fetch-json", "write-dir", "write-json", "command-fetch",
              "command-write", "out"):
        c.add_argument("--" + x, required=True)
    c.add_argument("--copy-mb", type=int, required=True)
    a = ap.parse_args(argv)
    text = {"trace": trace_summary, "counters": counters_summary,
            "stats": stats_summary}[a.kind](a)
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    sys.exit(main())
