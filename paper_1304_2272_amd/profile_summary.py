"""Summaries of rocprofv3 output for ``profiles/`` (measurement tooling; the
library does not use it).

``trace``    Markdown table of a ``--kernel-trace --stats`` run (its
             kernel_stats.csv, or a rocpd2summary markdown table).
``traffic``  HBM bytes of the triangular product from two ``--pmc`` runs
             (FETCH_SIZE, then WRITE_SIZE, both in KiB per dispatch), each
             scaled by what the same counter reads for a plain element-wise
             kernel of known size in the same run (``torch.bitwise_not`` over
             ``--copy-bytes`` bytes: it reads and writes that many bytes).
             Writes a JSON record that bench.py reports as ``roofline.traffic``
             while the kernel's sources keep the recorded SHA-256.

    python -m paper_1304_2272_amd.profile_summary traffic \\
        --fetch <FETCH_SIZE counter_collection.csv> --write <WRITE_SIZE csv> \\
        --kernel "trmm_stream_kernel<float, signed char" --copy-bytes 4294967296 \\
        --n 50000 --p 8 --columns 50000 --elem-bytes 4 --workload n50000_p8 \\
        --out profiles/trmm_fp32_n50000_p8_traffic.json
"""

from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join("paper_1304_2272_amd", "csrc")


def kernel_sources(kernel):
    """Source files (relative to the repository root) whose text decides the
    named kernel's code."""
    own = "sliced_kernels.hip" if ("sliced" in kernel or "paired" in kernel) else "trmm_kernels.hip"
    return [os.path.join(CSRC, own), os.path.join(CSRC, "trmm_common.h")]


def sources_sha256(paths):
    h = hashlib.sha256()
    for p in paths:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()


def _per_dispatch(path, counter):
    """{dispatch id: (kernel name, value)} for one counter of a CSV."""
    out = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = int(r["Dispatch_Id"])
        name, v = out.get(k, (r["Kernel_Name"], 0.0))
        out[k] = (name, v + float(r["Counter_Value"]))
    return out


def traffic(args):
    fetch = _per_dispatch(args.fetch, "FETCH_SIZE")
    write = _per_dispatch(args.write, "WRITE_SIZE")

    def split(d):
        copy = [v for name, v in d.values() if "bitwise_not" in name]
        kern = [v for name, v in d.values() if args.kernel in name]
        if not copy or not kern:
            raise SystemExit("copy probe or kernel dispatches missing from " + str(list(d.values())[:3]))
        # torch splits the element-wise kernel into several dispatches
        return sum(copy) * 1024.0, [v * 1024.0 for v in kern]

    fc, fk = split(fetch)
    wc, wk = split(write)
    f_cal = args.copy_bytes / fc
    w_cal = args.copy_bytes / wc
    launches = len(fk)
    fetch_b = sum(fk) * f_cal
    write_b = sum(wk) * w_cal
    n_pad = (args.n + 255) // 256 * 256
    # algorithmic bytes of the launches: the lower half of L^-1 once per
    # launch, every dosage byte once, the float64 partial sums once
    part_rows = args.part_rows
    alg = launches * (n_pad * (n_pad + 1) / 2 * args.elem_bytes) + args.columns * (
        args.n * args.x_bytes + 8 * (n_pad // part_rows))
    rec = {
        "kernel": args.kernel,
        "workload": args.workload,
        "launches": launches,
        "columns": args.columns,
        "fetch_bytes": fetch_b,
        "write_bytes": write_b,
        "traffic_bytes_per_launch": (fetch_b + write_b) / launches,
        "algorithmic_bytes_per_launch": alg / launches,
        "fetch_calibration": f_cal,
        "write_calibration": w_cal,
        "kernel_sources": kernel_sources(args.kernel),
        "kernel_source_sha256": sources_sha256(kernel_sources(args.kernel)),
    }
    json.dump(rec, open(args.out, "w"), indent=1)
    print(json.dumps(rec, indent=1))


def _short(name):
    for a, b in (("(gwas::TrmmArgs)", ""), ("(gwas::SolveArgs)", ""), ("(gwas::BandArgs)", ""),
                 ("(anonymous namespace)::", ""), ("bool _Accum", "__bf16")):
        name = name.replace(a, b)
    return name if len(name) <= 100 else name[:97] + "..."


def trace(args):
    data = []
    if args.stats.endswith(".csv"):
        # rocprofv3 --stats --output-format csv: <prefix>_kernel_stats.csv
        for r in csv.DictReader(open(args.stats)):
            data.append((_short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]),
                         float(r["Percentage"]), float(r["MinNs"]), float(r["MaxNs"])))
        data.sort(key=lambda d: -d[2])
    else:
        rows = [l for l in open(args.stats) if l.startswith("|")]
        for l in rows[2:]:
            c = [x.strip() for x in l.strip("|\n").split("|")]
            data.append((_short(c[0]), int(c[1]), float(c[2]), float(c[3]), float(c[4]), float(c[5]), float(c[6])))
    with open(args.out, "w") as f:
        f.write(f"# {args.title}\n\nCommand (repository root, one MI355X):\n\n```\n{args.command}\n```\n\n")
        f.write("`rocprofv3 --kernel-trace --stats`; times in ms, kernels by total time.\n\n")
        f.write("| kernel | calls | total ms | avg ms | % | min ms | max ms |\n|---|---:|---:|---:|---:|---:|---:|\n")
        for d in data[:args.top]:
            f.write(f"| `{d[0]}` | {d[1]} | {d[2] / 1e6:.1f} | {d[3] / 1e6:.3f} | {d[4]:.1f} | "
                    f"{d[5] / 1e6:.3f} | {d[6] / 1e6:.3f} |\n")
    print(open(args.out).read())


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--n", type=int, required=True)
    t.add_argument("--p", type=int, required=True)
    t.add_argument("--columns", type=int, required=True)
    t.add_argument("--elem-bytes", type=int, required=True)
    t.add_argument("--x-bytes", type=int, default=1)
    t.add_argument("--part-rows", type=int, default=64)
    t.add_argument("--workload", required=True)
    t.add_argument("--out", required=True)
    r = sub.add_parser("trace")
    r.add_argument("--stats", required=True,
                   help="kernel stats: rocprofv3's <prefix>_kernel_stats.csv, or a rocpd2summary -f md table")
    r.add_argument("--title", required=True)
    r.add_argument("--command", required=True)
    r.add_argument("--top", type=int, default=14)
    r.add_argument("--out", required=True)
    a = ap.parse_args()
    {"traffic": traffic, "trace": trace}[a.cmd](a)


if __name__ == "__main__":
    main()
