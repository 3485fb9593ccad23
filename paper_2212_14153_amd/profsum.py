"""Short text summaries of rocprofv3 output (kernel-trace statistics and HBM counters).

  python -m paper_2212_14153_amd.profsum trace --stats DIR/x_kernel_stats.csv \\
      --command "..." [--bench-json LINE_FILE] --out SUMMARY.md
  python -m paper_2212_14153_amd.profsum traffic --fetch FETCH.csv --write WRITE.csv \\
      --kernel step_kernel --storage f32 --workload c3 --nodes N --copy-bytes B \\
      --command "..." --out TRAFFIC.json

`traffic` turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of a kernel into HBM bytes per
launch, each scaled by what the same counter reads for the plain copy kernel of known size
that the same run dispatches (a copy of B bytes reads B and writes B bytes).  The JSON keeps
one entry per storage format, the workload it was measured on and the hash of the library
sources the counters were taken on, so a later change of the kernels or the layout
invalidates them.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import statistics

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_KERNEL = "copy_kernel"


def kernel_source_hash() -> str:
    """Hash of every kernel and runtime source (the memory layout is set by the runtime)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp", ".h")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """'void fpd::step_kernel<1, 1>(fpd::StepArgs)' -> 'step_kernel<1, 1>'."""
    name = re.sub(r"^void\s+", "", name)
    name = name.split("(")[0]
    return name.replace("fpd::", "")


def read_stats(path: str):
    with open(path, newline="") as f:
        rows = list(csv.DictReader(f))
    out = []
    for r in rows:
        out.append({"name": short_name(r["Name"]), "calls": int(r["Calls"]),
                    "total_ns": float(r["TotalDurationNs"]), "avg_ns": float(r["AverageNs"]),
                    "pct": float(r["Percentage"]), "min_ns": float(r["MinNs"]),
                    "max_ns": float(r["MaxNs"])})
    return out


def trace_summary(stats_csv: str, command: str, bench_json: str | None = None) -> str:
    rows = read_stats(stats_csv)
    lines = ["# rocprofv3 kernel-trace statistics", "", "Command:", "", "```",
             command, "```", "",
             "| kernel | calls | avg us | min us | max us | total ms | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{r['name']}` | {r['calls']} | {r['avg_ns'] / 1e3:.2f} | "
                     f"{r['min_ns'] / 1e3:.2f} | {r['max_ns'] / 1e3:.2f} | "
                     f"{r['total_ns'] / 1e6:.2f} | {r['pct']:.2f} |")
    if bench_json:
        with open(bench_json) as f:
            line = [ln for ln in f if ln.lstrip().startswith("{")][-1]
        rec = json.loads(line)
        lines += ["", "Figures of the same run, measured by the program itself with HIP events:", ""]
        roof = rec.get("roofline") or {}
        keep = {"value": rec.get("value"), "unit": rec.get("unit"),
                "ms_per_step": rec.get("ms_per_step"), "dtype": rec.get("dtype"),
                "kernel": roof.get("kernel"), "avg_launch_ms": roof.get("avg_launch_ms"),
                "achieved_GBps": roof.get("achieved"), "frac": roof.get("frac")}
        for k, v in keep.items():
            if v is not None:
                lines.append(f"- {k}: {v}")
    return "\n".join(lines) + "\n"


def read_counter(path: str, counter: str):
    """{kernel short name: [value per dispatch]} of one counter."""
    out = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            out.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def _pick(per_kernel: dict, key: str):
    vals = [v for k, vs in per_kernel.items() if key in k for v in vs]
    if not vals:
        raise SystemExit(f"no dispatch of a kernel matching {key!r} in the counter file")
    return vals


def traffic_entry(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int):
    """Scaled HBM bytes per launch of `kernel`; 'a+b' names the kernels of one pass (a
    split step's fluid and fiber kernels), whose per-dispatch medians add up."""
    fetch = read_counter(fetch_csv, "FETCH_SIZE")
    write = read_counter(write_csv, "WRITE_SIZE")
    copy_f = statistics.median(_pick(fetch, COPY_KERNEL)) * 1024.0
    copy_w = statistics.median(_pick(write, COPY_KERNEL)) * 1024.0
    f_fetch = copy_bytes / copy_f
    f_write = copy_bytes / copy_w
    parts = kernel.split("+")
    k_f = sum(statistics.median(_pick(fetch, k)) for k in parts) * 1024.0
    k_w = sum(statistics.median(_pick(write, k)) for k in parts) * 1024.0
    read, wrote = round(k_f * f_fetch), round(k_w * f_write)
    return {"fetch_factor": round(f_fetch, 4), "write_factor": round(f_write, 4),
            "read_bytes_per_launch": read, "write_bytes_per_launch": wrote,
            "bytes_per_launch": read + wrote,
            "dispatches": [min(len(_pick(fetch, k)) for k in parts),
                           min(len(_pick(write, k)) for k in parts)]}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--stats", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--bench-json")
    t.add_argument("--out", required=True)
    c = sub.add_parser("traffic")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--kernel", default="step_kernel")
    c.add_argument("--storage", required=True)
    c.add_argument("--workload", default="c3", help="bench.py --workload of the counted runs")
    c.add_argument("--nodes", type=int, required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--md", help="also append a readable line to this markdown file")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        text = trace_summary(a.stats, a.command, a.bench_json)
        with open(a.out, "w") as f:
            f.write(text)
        return
    ent = traffic_entry(a.fetch, a.write, a.kernel, a.copy_bytes)
    ent.update(nodes=a.nodes, kernel=a.kernel, workload=a.workload, command=a.command)
    try:
        with open(a.out) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    sha = kernel_source_hash()
    if rec.get("kernel_sha") != sha:
        rec = {"kernel_sha": sha, "entries": {}}
    rec["entries"][a.storage] = ent
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    if a.md:
        new = not os.path.exists(a.md)
        with open(a.md, "a") as f:
            if new:
                f.write("# HBM traffic of the lattice pass (rocprofv3 counters)\n\n"
                        "FETCH_SIZE and WRITE_SIZE per dispatch (median; for a split step "
                        "the fluid and the fiber kernel added), each scaled by the factor "
                        "that makes the same counter read the known size of a 1 GiB plain "
                        "copy dispatched in the same run.\n\n")
            f.write(f"## {a.storage}, {a.nodes} nodes, {a.kernel}, kernel source {sha}\n\n"
                    f"Commands (FETCH_SIZE, then WRITE_SIZE):\n\n```\n{a.command}\n```\n\n"
                    f"- fetch factor {ent['fetch_factor']}, write factor {ent['write_factor']}\n"
                    f"- read {ent['read_bytes_per_launch']} B, write "
                    f"{ent['write_bytes_per_launch']} B, total {ent['bytes_per_launch']} B "
                    f"per launch ({ent['dispatches'][0]} dispatches)\n\n")


if __name__ == "__main__":
    main()
