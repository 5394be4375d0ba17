#!/usr/bin/env python3
"""Throughput of the GLS-GWAS hot path on one MI355X.

A step is one gwas_stream_block call over one batch of SNPs already resident
in HBM (int8 dosages, the n = 50,000, p = 8 workload by default): the
triangular product L^-1 X_blk, the SNP cross products, the p x p solves and
the FP64 refinement, with b, var and info written to device memory.  The
context (Cholesky of M, inverse factor, whitened X_L and y) is built before
the timed region and its time is reported as ``init_s``.

Legs: ``fp32`` (reduced-precision product with FP64 accumulation and
refinement; this is ``value``), ``fp64`` (plain float64 path) and ``bf16``.
Errors of the reduced-precision legs are measured against the fp64 leg on the
same SNPs.  One JSON line goes to stdout.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SNP GLS solves/sec at n=50k,p=8 (mixed vs FP64); TRSM % of MFMA peak"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "int8": 5000.0}   # dense matrix-core peaks
PROBE_ITERS = 100000   # runs of 8 instructions per wave in the measured-peak probe
SLICES = 6   # int8 digits per entry of L^-1 in the int8 leg
WORKLOADS = {
    "n50000_p8": dict(n=50_000, p=8, m=1_000_000, step=50_000, x_dtype="i8"),
    "n20000_p4": dict(n=20_000, p=4, m=500_000, step=50_000, x_dtype="f64"),
    "n10000_p4": dict(n=10_000, p=4, m=100_000, step=50_000, x_dtype="f64"),
    "n1000_p4": dict(n=1_000, p=4, m=10_000, step=10_000, x_dtype="f64"),
    # n = 10^5, the largest n of the paper's measurements: M (80 GB) stays in
    # host memory so that the device holds the library's workspace (220 GB in
    # float32, 240 GB with int8 slices)
    "n100000_p8": dict(n=100_000, p=8, m=1_000_000, step=16_384, x_dtype="i8", m_host=True),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def normwise(b, bref):
    import torch
    d = (b - bref).reshape(b.shape[0], -1).norm(dim=1)
    r = bref.reshape(b.shape[0], -1).norm(dim=1)
    return float((d / r).max())


def measured_traffic(leg, workload_name):
    """HBM bytes per full launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None once the kernel source has changed."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"trmm_{leg}_{workload_name}_traffic.json")
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec.get("kernel_sources", []):
        full = os.path.join(ROOT, src)
        if not os.path.exists(full):
            return None, "kernel changed since the counters were taken"
        h.update(open(full, "rb").read())
    if not rec.get("kernel_sources") or rec.get("kernel_source_sha256") != h.hexdigest():
        return None, "kernel changed since the counters were taken"
    return rec["traffic_bytes_per_launch"], (
        f"FETCH_SIZE+WRITE_SIZE per launch over the {rec['launches']} launches of one step, calibrated on a "
        f"plain element-wise kernel; algorithmic {rec['algorithmic_bytes_per_launch']:.3g} B per launch")


def cpu_baseline(workload, seed, n_s, m_s, threads):
    """The oracle on a bounded sample of the workload: its first n_s
    individuals and m_s SNPs.  Its per-SNP cost is two triangular solves with
    the LU factors of M (2 n^2 flops each), so SNPs/s is scaled by (n_s/n)^2."""
    from threadpoolctl import threadpool_limits
    from oracle import GLSOracle
    from paper_1304_2272_amd import synth
    n, p = workload["n"], workload["p"]
    prob = synth.make_problem(n_s, p, seed)
    XR = synth.snp_block(n_s, seed, 0, m_s, dtype=np.float64)
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        orc = GLSOracle(prob["M"], prob["XL"], prob["Y"])
        t1 = time.perf_counter()
        orc.solve(XR)
        t2 = time.perf_counter()
    rate_s = m_s / (t2 - t1)
    scale = (n_s / n) ** 2
    return {
        "value": rate_s * scale, "unit": "SNP/s", "cores": threads, "kind": "oracle",
        "sample": (f"oracle on the same recipe restricted to the first {n_s} individuals and "
                   f"{m_s} SNPs ({rate_s:.1f} SNP/s measured there), scaled by (n_s/n)^2 = "
                   f"{scale:.4g} for its O(n^2) per-SNP solves; the one-off LU of M "
                   f"({t1 - t0:.2f} s at n_s) is excluded"),
        "measured_snps_per_s_at_sample": rate_s, "factor_s_at_sample": t1 - t0,
    }


def pinned_h2d_peak(nbytes=1 << 30, reps=3):
    """Host-to-device rate of one large copy from pinned host memory (GB/s),
    the roof of the PCIe-inclusive path."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src, non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    rate = nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return rate


def run_leg(name, prob_dev, blocks, steps, warmup, workload, pcie_steps=0):
    import torch
    from paper_1304_2272_amd import binding
    n = workload["n"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = binding.GwasContext(prob_dev["M"], prob_dev["XL"], prob_dev["Y"], precision=name,
                              x_dtype=workload["x_dtype"], slices=SLICES if name == "int8" else 0)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    outs = []
    for s in range(warmup):
        ctx.stream_block(blocks[s % len(blocks)])
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        b, var, info = ctx.stream_block(blocks[(warmup + s) % len(blocks)])
        outs.append(b)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, kms, kcols = ctx.kernel_time()
    info_bad = int((info != 0).sum())
    pcie = None
    if pcie_steps:
        # the same blocks handed over in pinned host memory: PCIe-inclusive rate
        host = [blocks[s % len(blocks)].cpu().pin_memory() for s in range(pcie_steps)]
        out = (torch.empty((host[0].shape[0], 1, workload["p"]), dtype=torch.float64).pin_memory(),
               torch.empty(host[0].shape[0], dtype=torch.float64).pin_memory(),
               torch.empty(host[0].shape[0], dtype=torch.int32).pin_memory())
        ctx.stream_block(host[0], out=out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for h in host:
            ctx.stream_block(h, out=out)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        nb = sum(h.numel() * h.element_size() for h in host)
        pcie = {"snps_per_s": sum(h.shape[0] for h in host) / el, "host_to_device_GBps": nb / el / 1e9,
                "pinned_h2d_peak_GBps": pinned_h2d_peak(),
                "steps": pcie_steps, "note": "dosages in pinned host memory, b/var/info to pinned host memory"}
        log(f"[{name}] PCIe-inclusive: {pcie['snps_per_s']:.1f} SNP/s, {pcie['host_to_device_GBps']:.1f} GB/s of dosages")
    ctx.close()
    snps = sum(blocks[(warmup + s) % len(blocks)].shape[0] for s in range(steps))
    ops_per_snp = float(n) * float(n) * (SLICES if name == "int8" else 1)
    achieved = ops_per_snp * kcols / (kms * 1e-3) / 1e12 if kms > 0 else 0.0
    fp64_equiv = float(n) * float(n) * kcols / (kms * 1e-3) / 1e12 if kms > 0 else 0.0
    peak = PEAK_TFLOPS[name]
    # the same instruction's rate measured on this device at its clock under load
    measured_peak = binding.peak_probe(name, iters=PROBE_ITERS) / 1e12
    log(f"[{name}] init {init_s:.2f} s, {snps} SNPs in {elapsed:.3f} s = {snps / elapsed:.1f} SNP/s, "
        f"TRMM {launches} launches {kms:.1f} ms -> {achieved:.2f} T{'OP' if name == 'int8' else 'FLOP'}/s "
        f"({achieved / peak:.3f} of peak, {achieved / measured_peak:.3f} of the measured {measured_peak:.1f})")
    return {
        "snps_per_s": snps / elapsed, "elapsed_s": elapsed, "init_s": init_s, "snps": snps,
        "ms_per_step": 1e3 * elapsed / max(steps, 1),
        "kernel": {"launches": launches, "total_ms": kms, "avg_ms": kms / max(launches, 1),
                   "columns": kcols},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak,
                     "unit": "TOP/s" if name == "int8" else "TFLOP/s", "frac": achieved / peak,
                     "measured_peak": measured_peak, "frac_of_measured": achieved / measured_peak},
        "n2_tflops": fp64_equiv,
        "rank_flags_last_step": info_bad,
        "pcie": pcie,
    }, outs


def run_cohorts(args):
    """Eight cohorts of uneven n (2k..30k), h^2 ~ U(0.2, 0.8), t = 64 traits,
    p = 4, sharing SNP positions with cohort-specific int8 dosages; a step is
    one block of SNP positions solved for every cohort and trait."""
    import torch
    from paper_1304_2272_amd import binding, synth
    binding.load()
    dev = torch.device("cuda:0")
    p, t, step = 4, 64, args.step_snps or 16384
    spec = synth.cohorts(8, args.seed)
    log("cohorts n =", [c["n"] for c in spec], "h2 =", [round(c["h2"], 3) for c in spec])
    data = []
    for i, c in enumerate(spec):
        pr = synth.make_problem(c["n"], p, c["seed"], t=t, h2=c["h2"], device="cuda:0")
        data.append({"M": pr["M"], "XL": torch.from_numpy(pr["XL"]).to(dev),
                     "Y": torch.from_numpy(pr["Y"]).to(dev), "n": c["n"],
                     "X": [synth.snp_block_device(c["n"], args.seed, s * step, step, dev, cohort=i)
                           for s in range(args.warmup + args.steps)]})
    torch.cuda.synchronize()
    n2 = sum(float(d["n"]) ** 2 for d in data)
    legs = {}
    outs = {}
    for leg, precision, grouped in [("fp64_grouped", "fp64", True), ("fp64_sequential", "fp64", False),
                                    ("fp32_grouped", "fp32", True), ("int8_grouped", "int8", True)]:
        t0 = time.perf_counter()
        ctxs = [binding.GwasContext(d["M"], d["XL"], d["Y"], precision=precision, x_dtype="i8",
                                    slices=SLICES if precision == "int8" else 0) for d in data]
        torch.cuda.synchronize()
        init_s = time.perf_counter() - t0
        def one(s):
            if grouped:
                return binding.stream_group(ctxs, [d["X"][s] for d in data])
            return [c.stream_block(d["X"][s]) for c, d in zip(ctxs, data)]
        for s in range(args.warmup):
            one(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [one(args.warmup + s) for s in range(args.steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        for c in ctxs:
            c.close()
        outs[leg] = res
        rate = args.steps * step * len(data) / el
        tflops = n2 * step * args.steps / el / 1e12
        legs[leg] = {"cohort_snps_per_s": rate, "trait_solves_per_s": rate * t, "init_s": init_s,
                     "ms_per_step": 1e3 * el / args.steps, "n2_tflops_whole_step": tflops}
        log(f"[{leg}] init {init_s:.2f} s; {rate:.1f} cohort-SNP/s ({rate * t:.3g} trait solves/s), "
            f"{tflops:.1f} TFLOP/s of triangular products over the whole step")
    errs = {}
    for leg in ("fp32_grouped", "int8_grouped"):
        errs[leg] = max(normwise(outs[leg][s][c][0], outs["fp64_grouped"][s][c][0])
                        for s in range(args.steps) for c in range(len(data)))
    seq_same = all(torch.equal(outs["fp64_sequential"][s][c][0], outs["fp64_grouped"][s][c][0])
                   for s in range(args.steps) for c in range(len(data)))
    log("errors vs fp64:", errs, "grouped == sequential bitwise:", seq_same)
    main = legs["fp32_grouped"]
    line = {
        "metric": "cohort-SNP GLS solves/sec, 8 cohorts n~U(2k,30k), t=64 traits, p=4",
        "value": main["cohort_snps_per_s"], "unit": "cohort-SNP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "cohorts8_t64", "cohort_n": [d["n"] for d in data], "p": p, "t": t,
                   "snps_per_step": step, "x_dtype": "int8", "precision": "fp32",
                   "inputs": "device-resident", "parallelism": "single GPU"},
        "legs": legs, "err_vs_fp64": errs, "grouped_equals_sequential": seq_same,
    }
    print(json.dumps(line), flush=True)


def run_gradient(args):
    """n = 10,000, p = 4, m = 10^5 float64 dosages: forward solves and the
    reverse pass of l = sum_i b_SNP,i^2 / var_i (dl/dy and dl/dh^2)."""
    import torch
    from paper_1304_2272_amd import binding, synth
    binding.load()
    n, p, m, step = 10_000, 4, 100_000, args.step_snps or 50_000
    dev = torch.device("cuda:0")
    prob = synth.make_problem(n, p, args.seed, device="cuda:0")
    M, XL, Y = prob["M"], torch.from_numpy(prob["XL"]).to(dev), torch.from_numpy(prob["Y"]).to(dev)
    blocks = [synth.snp_block_device(n, args.seed, s * step, step, dev, dtype=torch.float64)
              for s in range(m // step)]
    ctx = binding.GwasContext(M, XL, Y)
    ctx.stream_block(blocks[0][:1024])
    ctx.backward_begin()          # forms M^-1 and W once (reported as part of init)
    torch.cuda.synchronize()
    res = {}
    for rep in range(1 + args.warmup):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = [ctx.stream_block(X) for X in blocks]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.backward_begin()
        for X, (b, var, info) in zip(blocks, outs):
            bs = b[:, 0, :]
            gb = torch.zeros_like(bs)
            gb[:, -1] = 2.0 * bs[:, -1] / var
            gv = -(bs[:, -1] / var) ** 2
            ctx.backward_block(X, bs, var, info, gb, gv)
        gy, tr, ip = ctx.backward_end(torch.empty(n, dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = {"forward_s": t1 - t0, "backward_s": t2 - t1}
    ctx.close()
    h2 = prob["h2"]
    loss = float(sum(((b[:, 0, -1] ** 2) / var).sum() for b, var, _ in outs))
    dh2 = (ip - prob["sigma2"] * tr) / h2
    fwd = m / res["forward_s"]
    both = m / (res["forward_s"] + res["backward_s"])
    log(f"[grad] forward {fwd:.1f} SNP/s, forward+reverse {both:.1f} SNP/s; loss {loss:.6e} dl/dh2 {dh2:.6e}")
    line = {
        "metric": "SNP GLS solves/sec with gradient, n=10k, p=4 (forward + reverse pass)",
        "value": both, "unit": "SNP/s", "n_gpus": 1, "steps": m // step, "warmup": args.warmup,
        "ms_per_step": 1e3 * (res["forward_s"] + res["backward_s"]) / (m // step),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "n10000_p4_grad", "n": n, "p": p, "m": m, "x_dtype": "f64",
                   "loss": "sum_i b_SNP^2 / var", "inputs": "device-resident", "parallelism": "single GPU"},
        "forward_snps_per_s": fwd, "forward_s": res["forward_s"], "backward_s": res["backward_s"],
        "loss": loss, "dl_dh2": dh2, "dl_dy_norm": float(gy.norm()),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n50000_p8",
                    choices=sorted(WORKLOADS) + ["cohorts8_t64", "n10000_p4_grad"])
    ap.add_argument("--legs", default="fp32,fp64,int8,bf16")
    ap.add_argument("--fp64-steps", type=int, default=4)
    ap.add_argument("--bf16-steps", type=int, default=2)
    ap.add_argument("--int8-steps", type=int, default=4)
    ap.add_argument("--pcie-steps", type=int, default=2,
                    help="blocks streamed from pinned host memory after the timed steps (main leg)")
    ap.add_argument("--step-snps", type=int, default=0)
    ap.add_argument("--seed", type=int, default=1306)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=8192)
    ap.add_argument("--cpu-snps", type=int, default=8192)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "cohorts8_t64":
        run_cohorts(args)
        return
    if args.workload == "n10000_p4_grad":
        run_gradient(args)
        return

    import torch
    from paper_1304_2272_amd import binding, synth
    binding.load()
    w = dict(WORKLOADS[args.workload])
    if args.step_snps:
        w["step"] = args.step_snps
    n, p, step = w["n"], w["p"], w["step"]
    dev = torch.device("cuda:0")
    legs = [x for x in args.legs.split(",") if x]
    main_leg = legs[0]

    t0 = time.perf_counter()
    log(f"generating n={n} p={p} on {dev} ...")
    prob = synth.make_problem(n, p, args.seed, device="cuda:0")
    if w.get("m_host"):
        M_host = prob.pop("M").cpu()
        torch.cuda.empty_cache()
        prob_dev = {"M": M_host, "XL": prob["XL"], "Y": prob["Y"]}
    else:
        prob_dev = {"M": prob["M"], "XL": torch.from_numpy(prob["XL"]).to(dev),
                    "Y": torch.from_numpy(prob["Y"]).to(dev)}
    nblk = args.warmup + max(args.steps, args.fp64_steps, args.bf16_steps, args.int8_steps)
    xdt = torch.int8 if w["x_dtype"] == "i8" else torch.float64
    blocks = [synth.snp_block_device(n, args.seed, i * step, step, dev, dtype=xdt) for i in range(nblk)]
    torch.cuda.synchronize()
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s ({nblk} blocks of {step} SNPs)")

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.bitwise_not(src, out=dst)      # one element-wise kernel: reads and writes nb bytes
        torch.cuda.synchronize()
        log(f"copy probe: {nb} bytes read and written")
        del src, dst

    steps_of = {"fp32": args.steps, "fp64": args.fp64_steps, "bf16": args.bf16_steps,
                "int8": args.int8_steps}
    steps_of[main_leg] = args.steps
    res, outs = {}, {}
    for leg in legs:
        res[leg], outs[leg] = run_leg(leg, prob_dev, blocks, steps_of[leg], args.warmup, w,
                                      pcie_steps=args.pcie_steps if leg == main_leg else 0)
    errs = {}
    if "fp64" in outs:
        for leg in legs:
            if leg == "fp64":
                continue
            k = min(len(outs[leg]), len(outs["fp64"]))
            if k:
                errs[leg] = max(normwise(outs[leg][i], outs["fp64"][i]) for i in range(k))
                log(f"[{leg}] max normwise error vs fp64 over {k} steps: {errs[leg]:.3e}")
    del outs, blocks
    torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        try:
            threads = min(16, len(os.sched_getaffinity(0)))
        except AttributeError:
            threads = min(16, os.cpu_count() or 1)
        cn = min(args.cpu_n, n)
        log(f"cpu baseline: oracle at n_s={cn}, {args.cpu_snps} SNPs, {threads} threads ...")
        cpu = cpu_baseline(w, args.seed, cn, args.cpu_snps, threads)
        log(f"cpu baseline {cpu['value']:.3f} SNP/s (scaled)")

    r = res[main_leg]
    traffic, traffic_note = measured_traffic(main_leg, args.workload)
    end_to_end = w["m"] / (r["init_s"] + w["m"] / r["snps_per_s"])
    line = {
        "metric": METRIC if (n, p) == (50_000, 8) else METRIC.replace("n=50k,p=8", f"n={n // 1000}k,p={p}"),
        "value": r["snps_per_s"],
        "unit": "SNP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16", "int8": "i8"}[main_leg],
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "p": p, "snps_per_step": step,
                   "x_dtype": "int8" if w["x_dtype"] == "i8" else "f64",
                   "precision": main_leg,
                   "inputs": ("dosages device-resident; M, X_L and y handed over in host memory" if w.get("m_host")
                              else "device-resident"),
                   "parallelism": "single GPU"},
        "roofline": dict(r["roofline"], traffic=traffic, traffic_note=traffic_note),
        "cpu_baseline": cpu,
        "init_s": {k: v["init_s"] for k, v in res.items()},
        "legs": {k: {"snps_per_s": v["snps_per_s"], "ms_per_step": v["ms_per_step"],
                     "roofline": v["roofline"], "n2_tflops": v["n2_tflops"], "kernel": v["kernel"],
                     "snps": v["snps"]}
                 for k, v in res.items()},
        "pcie_inclusive": r["pcie"],
        "err_vs_fp64": errs,
        "end_to_end_snps_per_s": end_to_end,
        "end_to_end_m": w["m"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
