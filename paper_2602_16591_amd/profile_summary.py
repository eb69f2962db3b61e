"""Summaries of rocprofv3 output for the committed profiles (profiles/*.md).

Reads the CSV files that `rocprofv3 --output-format csv` writes (searched recursively under the
given output directories) and writes one markdown file: a table per kernel and a machine-readable
JSON block that bench.py reads (valid only while the kernel sources hash to the recorded value).

  trace     --kernel-trace --stats: calls, average / min / max duration and share per kernel
  traffic   two --pmc runs (FETCH_SIZE, then WRITE_SIZE): HBM bytes per launch, each counter
            scaled by what it reads for a plain copy of a known size (bench.py --copy-mib)
  counters  one --pmc run of SQ counters: per-launch averages (LDS and VALU instructions, ...)

Usage (from the repository root):
  python -m paper_2602_16591_amd.profile_summary trace DIR --workload NAME --title T --command C --out F
  python -m paper_2602_16591_amd.profile_summary traffic --fetch DIR --write DIR --copy-mib 256 ...
  python -m paper_2602_16591_amd.profile_summary counters DIR ...
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
# the device code whose counters a summary holds; any change to its code voids them
KERNEL_SOURCES = ("kernels.hip", "kernels.hpp", "particles.hip", "device_common.hpp")


def code_only(text: str) -> str:
    """C++ source with comments removed and every run of blank space made one space (string
    and character literals kept), so that editing a comment leaves the hash unchanged."""
    token = re.compile(r'"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'|//[^\n]*|/\*.*?\*/', re.S)
    stripped = token.sub(lambda m: " " if m.group(0).startswith("/") else m.group(0), text)
    return " ".join(stripped.split())


def kernel_source_sha256() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), encoding="utf-8") as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()


def short_name(name: str) -> str:
    """`void pswfe::(anonymous namespace)::k_gather<float, 13, 11>(float4 const*, ...)` ->
    `k_gather<float, 13, 11>`; other kernels keep their name without the argument list."""
    m = re.search(r"\b(k_\w+)(<[^()]*>)?\s*\(", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name.split("(")[0].strip()


def _rows(directory: str, suffix: str):
    files = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {directory}")
    for path in files:
        with open(path, newline="") as f:
            yield from csv.DictReader(f)


def _col(row: dict, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return row[low[n.lower()]]
    raise KeyError(f"none of {names} in {list(row)}")


def trace_table(directory: str):
    """Per kernel (short name): calls, average, min and max duration (us) and share of the total,
    from the --stats CSV (kernel_stats.csv)."""
    acc = defaultdict(lambda: {"calls": 0, "total_ns": 0.0, "min_ns": float("inf"), "max_ns": 0.0})
    for r in _rows(directory, "kernel_stats.csv"):
        k = short_name(_col(r, "Name", "KernelName", "Kernel_Name"))
        a = acc[k]
        calls = int(float(_col(r, "Calls")))
        a["calls"] += calls
        a["total_ns"] += float(_col(r, "TotalDurationNs", "TotalDuration"))
        a["min_ns"] = min(a["min_ns"], float(_col(r, "MinNs", "Min")))
        a["max_ns"] = max(a["max_ns"], float(_col(r, "MaxNs", "Max")))
    total = sum(a["total_ns"] for a in acc.values()) or 1.0
    out = {}
    for k, a in acc.items():
        out[k] = {"calls": a["calls"], "avg_us": a["total_ns"] / max(a["calls"], 1) / 1e3,
                  "min_us": a["min_ns"] / 1e3, "max_us": a["max_ns"] / 1e3, "share": a["total_ns"] / total}
    return dict(sorted(out.items(), key=lambda kv: -kv[1]["share"]))


def counter_means(directory: str):
    """{counter: {kernel: (dispatches, mean value per dispatch)}} from counter_collection.csv,
    plus {counter: max value over dispatches of kernels not named k_*} (the calibration copy)."""
    vals = defaultdict(lambda: defaultdict(list))
    other_max = defaultdict(float)
    for r in _rows(directory, "counter_collection.csv"):
        name = _col(r, "Kernel_Name", "KernelName", "Name")
        k = short_name(name)
        c = _col(r, "Counter_Name", "CounterName")
        v = float(_col(r, "Counter_Value", "CounterValue"))
        d = _col(r, "Dispatch_Id", "DispatchId", "Correlation_Id")
        vals[c][k].append((d, v))
        if not k.startswith("k_"):
            other_max[c] = max(other_max[c], v)
    means = {}
    for c, per in vals.items():
        means[c] = {}
        for k, lst in per.items():
            by_dispatch = defaultdict(float)   # a counter may be reported per XCD / agent: summed per dispatch
            for d, v in lst:
                by_dispatch[d] += v
            means[c][k] = (len(by_dispatch), sum(by_dispatch.values()) / len(by_dispatch))
    return means, dict(other_max)


def _header(title, commands, note):
    lines = [f"# {title}", "", "Command(s), from the repository root with `TMPDIR=/tmp`; this summary was written by",
             "`python -m paper_2602_16591_amd.profile_summary` from their CSV output:", "", "```"]
    lines += commands
    lines += ["```", ""]
    if note:
        lines += [note, ""]
    lines += ["Kernel source sha256 (kernels.hip, kernels.hpp, particles.hip, device_common.hpp; code with "
              f"comments and blank space removed): `{kernel_source_sha256()}`", ""]
    return lines


def _json_block(blob):
    return ["Machine-readable (read by bench.py; valid only while the kernel source hash matches):", "",
            "```json", json.dumps(blob, indent=1), "```", ""]


def write_trace(args):
    t = trace_table(args.dir)
    lines = _header(args.title, args.command, args.note)
    lines += ["| kernel | calls | avg us | min us | max us | share % |", "|---|---:|---:|---:|---:|---:|"]
    for k, a in t.items():
        lines.append(f"| `{k}` | {a['calls']} | {a['avg_us']:.2f} | {a['min_us']:.2f} | {a['max_us']:.2f} | "
                     f"{100 * a['share']:.2f} |")
    lines.append("")
    blob = {"kernel_source_sha256": kernel_source_sha256(), "workload": args.workload,
            "avg_us": {k: round(a["avg_us"], 3) for k, a in t.items()}}
    lines += _json_block(blob)
    _write(args.out, lines)


def write_traffic(args):
    fetch, fmax = counter_means(args.fetch)
    write, wmax = counter_means(args.write)
    fk = fetch.get("FETCH_SIZE") or {}
    wk = write.get("WRITE_SIZE") or {}
    copy_bytes = args.copy_mib * (1 << 20)
    f_fac = copy_bytes / (fmax["FETCH_SIZE"] * 1024.0)
    w_fac = copy_bytes / (wmax["WRITE_SIZE"] * 1024.0)
    note = (f"Calibration: `--copy-mib {args.copy_mib}` copies a {args.copy_mib} MiB device buffer (a plain copy of known "
            f"traffic). Its largest dispatch reads FETCH_SIZE = {fmax['FETCH_SIZE']:.1f} KiB and WRITE_SIZE = "
            f"{wmax['WRITE_SIZE']:.1f} KiB for {copy_bytes // 1024} KiB read and written, so bytes = FETCH_SIZE x 1024 x "
            f"{f_fac:.4f} and WRITE_SIZE x 1024 x {w_fac:.4f}. Values are averages over all dispatches of the kernel "
            "(calibration and timed steps). " + (args.note or ""))
    lines = _header(args.title, args.command, note)
    lines += ["| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read bytes (calibrated) | written bytes | total MB |",
              "|---|---:|---:|---:|---:|---:|---:|"]
    per = {}
    for k in sorted(set(fk) & set(wk)):
        if not k.startswith("k_"):
            continue
        nd, f = fk[k]
        _, w = wk[k]
        rb, wb = f * 1024 * f_fac, w * 1024 * w_fac
        per[k] = int(round(rb + wb))
        lines.append(f"| `{k}` | {nd} | {f:.1f} | {w:.1f} | {rb:.0f} | {wb:.0f} | {(rb + wb) / 1e6:.3f} |")
    lines.append("")
    blob = {"kernel_source_sha256": kernel_source_sha256(), "workload": args.workload,
            "calibration": {"fetch_factor": f_fac, "write_factor": w_fac, "copy_mib": args.copy_mib},
            "bytes_per_launch": per}
    lines += _json_block(blob)
    _write(args.out, lines)


COUNTER_KEYS = {"SQ_INSTS_LDS": "lds_instr", "SQ_LDS_BANK_CONFLICT": "lds_bank_conflict_cycles",
                "SQ_INSTS_VALU": "valu_instr", "SQ_WAVES": "waves"}


def write_counters(args):
    means, _ = counter_means(args.dir)
    kernels = sorted({k for c in means.values() for k in c if k.startswith("k_")})
    cols = list(means)
    lines = _header(args.title, args.command, args.note)
    lines += ["| kernel | " + " | ".join(cols) + " |", "|---|" + "---:|" * len(cols)]
    per = {}
    for k in kernels:
        row = {}
        for c in cols:
            row[COUNTER_KEYS.get(c, c)] = means[c].get(k, (0, 0.0))[1]
        per[k] = row
        lines.append(f"| `{k}` | " + " | ".join(f"{means[c].get(k, (0, 0.0))[1]:.0f}" for c in cols) + " |")
    lines.append("")
    blob = {"kernel_source_sha256": kernel_source_sha256(), "workload": args.workload, "per_launch": per}
    lines += _json_block(blob)
    _write(args.out, lines)


def _write(path, lines):
    with open(path, "w") as f:
        f.write("\n".join(lines))
    print(f"wrote {path}")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    for name in ("trace", "traffic", "counters"):
        p = sub.add_parser(name)
        if name == "traffic":
            p.add_argument("--fetch", required=True)
            p.add_argument("--write", required=True)
            p.add_argument("--copy-mib", type=int, required=True)
        else:
            p.add_argument("dir")
        p.add_argument("--workload", required=True)
        p.add_argument("--title", required=True)
        p.add_argument("--command", action="append", required=True, help="the rocprofv3 command (repeatable)")
        p.add_argument("--note", default="")
        p.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    {"trace": write_trace, "traffic": write_traffic, "counters": write_counters}[args.what](args)


if __name__ == "__main__":
    main()
