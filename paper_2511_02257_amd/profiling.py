"""Summaries of rocprofv3 output for the committed profiles.

traffic: HBM bytes per launch of one kernel variant from two counter runs
(FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled by what the
same counter reads for a plain device copy of known size.  --grid keeps only
the dispatches of that grid size (several launch shapes of one kernel, e.g.
K32 and K33 launches of the same variant).  Entries for several variants of
the same kernel source accumulate in one file; a different source hash starts
the file afresh.

    python -m paper_2511_02257_amd.profiling traffic \\
        --kernel 'hec_mfma<double' --variant 23 --grid 901120 \\
        --fetch out/pmc_fetch/fetch_counter_collection.csv \\
        --write out/pmc_write/write_counter_collection.csv \\
        --copy-fetch out/pmc_copy_fetch/cf_counter_collection.csv \\
        --copy-write out/pmc_copy_write/cw_counter_collection.csv \\
        --copy-bytes 1073741824 --out profiles/hec_traffic_baryon_mix.json

dispatches: per (kernel, grid size) the calls and the average, minimum and
maximum duration from a rocprofv3 kernel trace (CSV), as a markdown table.

    python -m paper_2511_02257_amd.profiling dispatches out/prof/run_kernel_trace.csv
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _grid(r):
    for k in ("Grid_Size", "Grid_Size_X"):
        if k in r and r[k]:
            return int(r[k])
    return None


def _values(path, kernel_substr, grid=None):
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if kernel_substr in r["Kernel_Name"] and (grid is None or _grid(r) == grid):
                out.append(float(r["Counter_Value"]))
    return out


def dispatches(args):
    groups = {}
    with open(args.trace) as f:
        for r in csv.DictReader(f):
            key = (r["Kernel_Name"], _grid(r))
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            groups.setdefault(key, []).append(d)
    print("| Kernel | Grid | Calls | Average us | Min us | Max us |")
    print("|---|---|---|---|---|---|")
    for (name, grid), ds in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        short = name if len(name) < 90 else name[:87] + "..."
        print(f"| `{short}` | {grid} | {len(ds)} | {sum(ds) / len(ds):.1f} | {min(ds):.1f} | {max(ds):.1f} |")


def _code_only(text):
    """Source text without comments and with whitespace collapsed, so that an
    edit of a comment does not count as a change of the kernel."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_sha256():
    h = hashlib.sha256()
    for rel in ("paper_2511_02257_amd/csrc/kernels/kernels.hip", "paper_2511_02257_amd/csrc/kernels/hec.hpp",
                "paper_2511_02257_amd/csrc/kernels/hec_f64.hip", "paper_2511_02257_amd/csrc/kernels/desc.hpp"):
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def traffic(args):
    fetch = _values(args.fetch, args.kernel, args.grid)
    write = _values(args.write, args.kernel, args.grid)
    cf = _values(args.copy_fetch, args.copy_kernel)
    cw = _values(args.copy_write, args.copy_kernel)
    if not fetch or len(fetch) != len(write) or not cf or not cw:
        raise SystemExit("counter files do not match the kernel names")
    kib = args.copy_bytes / 1024.0
    kf = kib / (sum(cf) / len(cf))
    kw = kib / (sum(cw) / len(cw))
    per_launch = (sum(fetch) * kf + sum(write) * kw) * 1024.0 / len(fetch)
    entry = {
        "dispatches": len(fetch),
        "fetch_scale": round(kf, 5), "write_scale": round(kw, 5),
        "fetch_bytes_per_launch": sum(fetch) * kf * 1024.0 / len(fetch),
        "write_bytes_per_launch": sum(write) * kw * 1024.0 / len(write),
        "traffic_bytes_per_launch": per_launch,
    }
    sha = kernel_source_sha256()
    rec = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            rec = json.load(f)
    if rec.get("kernel_sha256") != sha or rec.get("kernel") != args.kernel:
        rec = {"kernel": args.kernel, "kernel_sha256": sha, "variants": {},
               "counters": "FETCH_SIZE and WRITE_SIZE (KiB per dispatch), separate rocprofv3 --pmc runs"}
    if args.grid is not None:
        entry["grid"] = args.grid
    rec["variants"][str(args.variant)] = entry
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--variant", type=int, required=True, help="kernel variant index (binding.variant_index)")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-kernel", default="copyBuffer")
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--out", required=True)
    t.add_argument("--grid", type=int, default=None, help="only dispatches of this grid size (work-items)")
    d = sub.add_parser("dispatches")
    d.add_argument("trace")
    args = ap.parse_args()
    if args.cmd == "traffic":
        traffic(args)
    elif args.cmd == "dispatches":
        dispatches(args)


if __name__ == "__main__":
    main()
