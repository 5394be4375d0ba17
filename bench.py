#!/usr/bin/env python3
"""Throughput of the GLS-GWAS hot path on one MI355X.

Default workload ``n50000_p8``: n = 50,000 individuals, p = 8, m = 10^6 SNPs
whose int8 dosages sit in pinned host memory as 20 distinct blocks of 50,000
SNPs.  A step is one block handed to the library with
``gwas_stream_block_async`` (Algorithm 2: host-to-device copy of the block,
triangular product L^-1 X_blk, SNP cross products, column dots, p x p solves)
with b, var and info written back to pinned host memory; the steps are queued
one after another and the timed region ends when ``gwas_stream_wait``
returns.  The context (Cholesky of M, inverse factor, whitened X_L and y) is
built before the timed region and reported as ``init_s``.

``value`` is the float64 path (``fp64``), the paper's arithmetic.  The other
legs run the same stream: ``fp32`` and ``bf16`` (reduced-precision product with
float64 refinement) and ``int8`` (int8 slices of L^-1 with exact int32 sums).
Their errors against the float64 leg cover every SNP: normwise over b_i, the
SNP coefficient in standard-error units (|db_SNP| / sqrt(var)) and relative,
and var.  Compact forms of the other four workloads (``n1000_p4``,
``n20000_p4`` streamed as float64 from pinned host memory, ``cohorts8_t64``,
``n10000_p4_grad``) run after it, and the CPU oracle is timed on one pinned
host core.  One JSON line goes to stdout.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SNP GLS solves/sec at n=50k,p=8 (mixed vs FP64); TRSM % of MFMA peak"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "int8": 5000.0,   # dense matrix-core peaks
               "bf16x3": 2500.0}
PROBE_KIND = {"bf16x3": "bf16"}   # instruction each leg runs, for the measured peak
PROBE_ITERS = 100000   # runs of 8 instructions per wave in the measured-peak probe
SLICES = 6             # int8 digits per entry of L^-1 in the int8 leg
DTYPE_NAME = {"fp64": "f64", "fp32": "f32", "bf16": "bf16", "int8": "i8", "bf16x3": "bf16x3"}
WORKLOADS = {
    "n50000_p8": dict(n=50_000, p=8, m=1_000_000, step=50_000, x_dtype="i8"),
    "n20000_p4": dict(n=20_000, p=4, m=500_000, step=5_000, x_dtype="f64"),
    "n10000_p4": dict(n=10_000, p=4, m=100_000, step=50_000, x_dtype="f64"),
    "n1000_p4": dict(n=1_000, p=4, m=10_000, step=10_000, x_dtype="f64"),
    # n = 10^5, the largest n of the paper's measurements: M (80 GB) stays in
    # host memory so that the device holds the library's workspace
    "n100000_p8": dict(n=100_000, p=8, m=1_000_000, step=16_384, x_dtype="i8", m_host=True),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class PinnedHost:
    """Page-locked host memory of exactly ``nbytes`` (hipHostMalloc through the
    HIP runtime torch has loaded), viewed as a numpy array; freed by close()."""

    def __init__(self, shape, dtype):
        import torch  # noqa: F401  (loads the HIP runtime the library shares)
        self._hip = ctypes.CDLL("libamdhip64.so.7")
        self._hip.hipHostMalloc.restype = ctypes.c_int
        self._hip.hipHostMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_uint]
        self._hip.hipHostFree.restype = ctypes.c_int
        self._hip.hipHostFree.argtypes = [ctypes.c_void_p]
        dt = np.dtype(dtype)
        nbytes = int(np.prod(shape)) * dt.itemsize
        ptr = ctypes.c_void_p()
        rc = self._hip.hipHostMalloc(ctypes.byref(ptr), max(nbytes, 1), 0)
        if rc != 0:
            raise MemoryError(f"hipHostMalloc({nbytes}) failed with {rc}")
        self.ptr = ptr.value
        buf = (ctypes.c_char * max(nbytes, 1)).from_address(self.ptr)
        self.array = np.frombuffer(buf, dtype=dt, count=int(np.prod(shape))).reshape(shape)

    def close(self):
        if self.ptr:
            self.array = None
            self._hip.hipHostFree(self.ptr)
            self.ptr = None


def snp_errors(b, var, info, bref, vref, iref):
    """Errors of (b, var) against the float64 leg over every SNP both solved:
    normwise over b_i; the SNP coefficient in standard-error units
    |db_SNP| / sqrt(var_ref) and relative |db_SNP| / |b_SNP,ref| (max, and
    the median since b_SNP has a zero mean); relative var."""
    ok = (info == 0) & (iref == 0)
    b, bref = b[ok].reshape(int(ok.sum()), -1), bref[ok].reshape(int(ok.sum()), -1)
    var, vref = var[ok], vref[ok]
    p = bref.shape[1]
    nw = np.linalg.norm(b - bref, axis=1) / np.linalg.norm(bref, axis=1)
    d = np.abs(b[:, p - 1] - bref[:, p - 1])
    se = d / np.sqrt(vref)
    rel = d / np.abs(bref[:, p - 1])
    vr = np.abs(var - vref) / vref
    return {"snps": int(ok.sum()), "info_mismatch": int((info != iref).sum()),
            "normwise_max": float(nw.max()), "snp_se_units_max": float(se.max()),
            "snp_rel_max": float(rel.max()), "snp_rel_median": float(np.median(rel)),
            "var_rel_max": float(vr.max())}


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
        f"FETCH_SIZE+WRITE_SIZE per launch over {rec['launches']} launches ({rec['columns']} SNP columns), "
        f"calibrated on a plain element-wise kernel; algorithmic {rec['algorithmic_bytes_per_launch']:.3g} B "
        f"per launch")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(workload, seed, n_s, m_s):
    """The plain C oracle (single-threaded float64, no BLAS) on one pinned
    host core, on a bounded sample of the workload (its first n_s
    individuals and m_s SNPs).  Its factorisation costs O(n^3) and each SNP
    two triangular solves with the Cholesky factor of M (O(n^2)), so the
    full-size figures are extrapolated from the sample: SNPs/s by
    (n_s/n)^2, the factorisation by (n/n_s)^3."""
    from oracle import GLSPlain
    from paper_1304_2272_amd import synth
    n, m = workload["n"], workload["m"]
    prob = synth.make_problem(n_s, workload["p"], seed)
    XR = synth.snp_block(n_s, seed, 0, m_s, dtype=np.float64)
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        orc = GLSPlain(prob["M"], prob["XL"], prob["Y"])
        t1 = time.perf_counter()
        orc.solve(XR)
        t2 = time.perf_counter()
    finally:
        os.sched_setaffinity(0, old)
    rate_s = m_s / (t2 - t1)
    rate = rate_s * (n_s / n) ** 2
    t_factor = (t1 - t0) * (n / n_s) ** 3
    return {
        "value": rate, "unit": "SNP/s", "cores": 1, "kind": "oracle",
        "sample": (f"plain C oracle (single-threaded float64, no BLAS, pinned to core {core}) on the same recipe "
                   f"restricted to the first {n_s} individuals and {m_s} SNPs: {rate_s:.1f} SNP/s there, "
                   f"scaled by (n_s/n)^2 = {(n_s / n) ** 2:.4g} for its O(n^2) per-SNP solves"),
        "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity_before": sorted(old),
        "measured_snps_per_s_at_sample": rate_s, "factor_s_at_sample": t1 - t0,
        "extrapolated_factor_s": t_factor,
        "extrapolated_end_to_end_s": t_factor + m / rate,
        "extrapolated_note": (f"extrapolated, not measured: factorisation {t1 - t0:.2f} s at n_s scaled by "
                              f"(n/n_s)^3, plus m = {m} SNPs at the scaled rate"),
    }


def pinned_h2d_peak(nbytes=1 << 30, reps=3):
    """Host-to-device rate of one large copy from pinned host memory (GB/s)."""
    import torch
    h = PinnedHost((nbytes,), np.uint8)
    src = torch.from_numpy(h.array)
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    rate = nbytes * reps / (time.perf_counter() - t0) / 1e9
    del src, dst
    h.close()
    return rate


def host_blocks(n, seed, step, count, dtype, dev, cohort=None):
    """`count` distinct SNP blocks of `step` columns in one pinned host buffer
    (count, step, n), drawn on the device and copied out."""
    import torch
    npdt = np.int8 if dtype == torch.int8 else np.float64
    buf = PinnedHost((count, step, n), npdt)
    t = torch.from_numpy(buf.array)
    for i in range(count):
        t[i].copy_(synthesize(n, seed, i * step, step, dev, dtype, cohort))
    return buf


def synthesize(n, seed, start, cols, dev, dtype, cohort=None):
    from paper_1304_2272_amd import synth
    return synth.snp_block_device(n, seed, start, cols, dev, dtype=dtype, cohort=cohort)


def stream_leg(name, prob_dev, blocks, steps, w, p, t=1):
    """Init a context, warm it up on one block, then queue `steps` host blocks
    with gwas_stream_block_async and wait.  Returns the leg's record and its
    outputs (pinned host arrays over every SNP)."""
    import torch
    from paper_1304_2272_amd import binding
    n = w["n"]
    nb, step = blocks.array.shape[0], blocks.array.shape[1]
    m = steps * step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = binding.GwasContext(prob_dev["M"], prob_dev["XL"], prob_dev["Y"], precision=name,
                              x_dtype=w["x_dtype"], slices=SLICES if name == "int8" else 0)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    out_b = PinnedHost((m, t, p), np.float64)
    out_v = PinnedHost((m,), np.float64)
    out_i = PinnedHost((m,), np.int32)
    ob, ov, oi = (torch.from_numpy(x.array) for x in (out_b, out_v, out_i))
    X = [torch.from_numpy(blocks.array[i]) for i in range(nb)]
    ctx.stream_block_async(X[0], (ob[:step], ov[:step], oi[:step]))   # warm-up, untimed
    ctx.wait()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for s in range(steps):
        sl = slice(s * step, (s + 1) * step)
        ctx.stream_block_async(X[s % nb], (ob[sl], ov[sl], oi[sl]))
    ctx.wait()
    elapsed = time.perf_counter() - t0
    launches, kms, kcols = ctx.kernel_time()
    ctx.close()
    # products per SNP: int8 digits of L^-1; bfloat16 slice pairs (three with
    # int8 dosages, six with float64 ones)
    mult = SLICES if name == "int8" else (3 if w["x_dtype"] == "i8" else 6) if name == "bf16x3" else 1
    ops_per_snp = float(n) * float(n) * mult
    achieved = ops_per_snp * kcols / (kms * 1e-3) / 1e12 if kms > 0 else 0.0
    peak = PEAK_TFLOPS[name]
    measured_peak = binding.peak_probe(PROBE_KIND.get(name, name), iters=PROBE_ITERS) / 1e12
    unit = "TOP/s" if name == "int8" else "TFLOP/s"
    log(f"[{name}] init {init_s:.2f} s, {m} SNPs from pinned host in {elapsed:.3f} s = {m / elapsed:.1f} SNP/s; "
        f"product {launches} launches, {kms / max(launches, 1):.2f} ms avg -> {achieved:.2f} {unit} "
        f"({achieved / peak:.3f} of peak, {achieved / measured_peak:.3f} of the measured {measured_peak:.1f})")
    rec = {
        "snps_per_s": m / elapsed, "elapsed_s": elapsed, "init_s": init_s, "snps": m,
        "ms_per_step": 1e3 * elapsed / steps,
        "host_to_device_GBps": m * n * blocks.array.itemsize / elapsed / 1e9,
        "kernel": {"launches": launches, "total_ms": kms, "avg_ms": kms / max(launches, 1), "columns": kcols},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "measured_peak": measured_peak,
                     "frac_of_measured": achieved / measured_peak},
        "n2_tflops": float(n) * float(n) * kcols / (kms * 1e-3) / 1e12 if kms > 0 else 0.0,
        "rank_flags": int((out_i.array != 0).sum()),
    }
    if name == "int8":
        rec["slices"] = SLICES
    return rec, (out_b, out_v, out_i)


def compact_c1(seed):
    """n = 1,000, p = 4, m = 10^4 float64 dosages from pinned host memory, one call."""
    import torch
    from paper_1304_2272_amd import binding, synth
    n, p, m = 1000, 4, 10_000
    dev = torch.device("cuda:0")
    prob = synth.make_problem(n, p, seed, device="cuda:0")
    blocks = host_blocks(n, seed, m, 1, torch.float64, dev)
    X = torch.from_numpy(blocks.array[0])
    with binding.GwasContext(prob["M"], torch.from_numpy(prob["XL"]).to(dev),
                             torch.from_numpy(prob["Y"]).to(dev)) as ctx:
        out = (torch.empty((m, 1, p), dtype=torch.float64).pin_memory(),
               torch.empty(m, dtype=torch.float64).pin_memory(), torch.empty(m, dtype=torch.int32).pin_memory())
        ctx.stream_block(X, out=out)
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.stream_block(X, out=out)
        el = time.perf_counter() - t0
    blocks.close()
    rate = reps * m / el
    log(f"[n1000_p4] {rate:.1f} SNP/s (float64 dosages from pinned host memory, {m} SNPs per call)")
    return {"snps_per_s": rate, "n": n, "p": p, "snps_per_call": m, "calls": reps, "precision": "fp64",
            "inputs": "float64 dosages in pinned host memory, outputs to pinned host memory"}


def compact_c2(seed, nblocks):
    """n = 20,000, p = 4: `nblocks` distinct float64 host blocks of 5,000 SNPs
    in pinned host memory, queued with gwas_stream_block_async."""
    import torch
    from paper_1304_2272_amd import synth
    n, p, step = 20_000, 4, 5_000
    dev = torch.device("cuda:0")
    w = dict(n=n, p=p, x_dtype="f64")
    prob = synth.make_problem(n, p, seed, device="cuda:0")
    prob_dev = {"M": prob["M"], "XL": torch.from_numpy(prob["XL"]).to(dev), "Y": torch.from_numpy(prob["Y"]).to(dev)}
    blocks = host_blocks(n, seed, step, nblocks, torch.float64, dev)
    rec, outs = stream_leg("fp64", prob_dev, blocks, nblocks, w, p)
    for o in outs:
        o.close()
    blocks.close()
    del prob_dev, prob
    torch.cuda.empty_cache()
    return {"snps_per_s": rec["snps_per_s"], "init_s": rec["init_s"], "snps": rec["snps"],
            "host_blocks": nblocks, "host_block_snps": step, "host_to_device_GBps": rec["host_to_device_GBps"],
            "kernel": rec["kernel"], "roofline": rec["roofline"], "precision": "fp64",
            "inputs": "float64 dosages (160 KB per SNP) in pinned host memory, queued blocks"}


def compact_c4(seed, steps, step=16384):
    """Eight cohorts of uneven n (2k..30k), h^2 ~ U(0.2, 0.8), t = 64 traits,
    p = 4, cohort-specific int8 dosages at shared positions (device
    resident); grouped launches (float64, and int8 slices) and per-context
    calls (float64) over `steps` blocks of positions."""
    import torch
    from paper_1304_2272_amd import binding, synth
    dev = torch.device("cuda:0")
    p, t = 4, 64
    spec = synth.cohorts(8, seed)
    data = []
    for i, c in enumerate(spec):
        pr = synth.make_problem(c["n"], p, c["seed"], t=t, h2=c["h2"], device="cuda:0")
        data.append({"M": pr["M"], "XL": torch.from_numpy(pr["XL"]).to(dev), "Y": torch.from_numpy(pr["Y"]).to(dev),
                     "n": c["n"], "X": [synthesize(c["n"], seed, s * step, step, dev, torch.int8, cohort=i)
                                        for s in range(steps + 1)]})
    torch.cuda.synchronize()
    legs, outs = {}, {}
    # (leg, precision, grouped, graph, SNP positions per call); calls of 512
    # positions run a 512-column sub-block context
    for leg, precision, grouped, graph, width in [
            ("fp64_grouped", "fp64", True, False, step), ("fp64_sequential", "fp64", False, False, step),
            ("int8_grouped", "int8", True, False, step), ("fp32_grouped", "fp32", True, False, step),
            ("fp32_grouped_graph_512", "fp32", True, True, 512), ("fp64_grouped_graph_512", "fp64", True, True, 512)]:
        t0 = time.perf_counter()
        ctxs = [binding.GwasContext(d["M"], d["XL"], d["Y"], precision=precision, x_dtype="i8",
                                    slices=SLICES if precision == "int8" else 0,
                                    dev_block=width if width < step else 0) for d in data]
        torch.cuda.synchronize()
        init_s = time.perf_counter() - t0

        def one(s):
            if width < step:    # the block's positions in calls of `width`
                return [binding.stream_group(ctxs, [d["X"][s][q:q + width] for d in data], graph=graph)
                        for q in range(0, step, width)]
            if grouped:
                return binding.stream_group(ctxs, [d["X"][s] for d in data], graph=graph)
            return [c.stream_block(d["X"][s]) for c, d in zip(ctxs, data)]
        one(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [one(1 + s) for s in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        for c in ctxs:
            c.close()
        if width == step:
            outs[leg] = res
        rate = steps * step * len(data) / el
        legs[leg] = {"cohort_snps_per_s": rate, "trait_solves_per_s": rate * t, "init_s": init_s,
                     "ms_per_step": 1e3 * el / steps, "snps_per_call": width, "graph": graph}
        log(f"[cohorts8_t64 {leg}] init {init_s:.2f} s; {rate:.1f} cohort-SNP/s ({rate * t:.3g} trait solves/s)")
        del res
    ref = outs["fp64_grouped"]
    err = max(float(((outs["int8_grouped"][s][c][0] - ref[s][c][0]).reshape(step, -1).norm(dim=1)
                     / ref[s][c][0].reshape(step, -1).norm(dim=1)).max())
              for s in range(steps) for c in range(len(data)))
    same = all(torch.equal(outs["fp64_sequential"][s][c][0], ref[s][c][0])
               for s in range(steps) for c in range(len(data)))
    del data, outs, ref
    torch.cuda.empty_cache()
    legs["fp32_512_vs_full_width"] = legs["fp32_grouped_graph_512"]["cohort_snps_per_s"] / \
        legs["fp32_grouped"]["cohort_snps_per_s"]
    return {"legs": legs, "cohort_n": [c["n"] for c in spec], "t": t, "p": p, "snps_per_step": step,
            "steps": steps, "int8_normwise_err_vs_fp64": err, "grouped_equals_sequential": same,
            "inputs": "int8 dosages device-resident"}


def compact_c5(seed, m=100_000, step=50_000):
    """n = 10,000, p = 4, m = 10^5 float64 dosages: the forward solves and the
    reverse pass of l = sum_i b_SNP,i^2 / var_i (dl/dy and dl/dh^2)."""
    import torch
    from paper_1304_2272_amd import binding, synth
    n, p = 10_000, 4
    dev = torch.device("cuda:0")
    prob = synth.make_problem(n, p, seed, device="cuda:0")
    M, XL, Y = prob["M"], torch.from_numpy(prob["XL"]).to(dev), torch.from_numpy(prob["Y"]).to(dev)
    blocks = [synthesize(n, seed, s * step, step, dev, torch.float64) for s in range(m // step)]
    res = {}
    with binding.GwasContext(M, XL, Y) as ctx:
        ctx.stream_block(blocks[0][:1024])
        ctx.backward_begin()          # forms M^-1 and W once (part of the set-up)
        for _ in range(2):            # the first pass warms up
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
            res = {"forward_s": t1 - t0, "backward_s": time.perf_counter() - t1}
    dh2 = (ip - prob["sigma2"] * tr) / prob["h2"]
    both = m / (res["forward_s"] + res["backward_s"])
    log(f"[n10000_p4_grad] forward {m / res['forward_s']:.1f} SNP/s, forward+reverse {both:.1f} SNP/s, "
        f"dl/dh2 {dh2:.6e}")
    del blocks, outs, M, XL, Y, prob
    torch.cuda.empty_cache()
    return {"snps_per_s_forward_and_reverse": both, "forward_snps_per_s": m / res["forward_s"],
            "forward_s": res["forward_s"], "backward_s": res["backward_s"], "m": m, "n": n, "p": p,
            "dl_dh2": dh2, "dl_dy_norm": float(gy.norm()), "loss": "sum_i b_SNP^2 / var",
            "inputs": "float64 dosages device-resident"}


def compact_banded(seed, widths, n=50_000, p=8, step=50_000, steps=2, x_dtype="i8"):
    """Banded M (relatives grouped near the diagonal, Section 5.1) at
    n = 50,000, p = 8: for each half-bandwidth w, dosages in pinned host
    memory queued as in the main legs (int8 by default; float64 dosages in
    blocks of 16,384 SNPs).  The algorithmic work of a banded forward
    substitution is 2 n w flops per SNP; with blocks of W = w rounded up to
    256 rows the kernels run 3.125 n_pad W (int8 dosages with W of 256 or
    512: one launch per sub-block, each wave's triangular part stopping at its
    own rows) or n_pad (3 W + 128) (one launch per block row)."""
    import torch
    from paper_1304_2272_amd import binding, synth
    dev = torch.device("cuda:0")
    if x_dtype == "f64":
        step = min(step, 16_384)
    blocks = host_blocks(n, seed, step, steps, torch.int8 if x_dtype == "i8" else torch.float64, dev)
    X = [torch.from_numpy(blocks.array[i]) for i in range(steps)]
    out_b = PinnedHost((step * steps, 1, p), np.float64)
    out_v = PinnedHost((step * steps,), np.float64)
    out_i = PinnedHost((step * steps,), np.int32)
    ob, ov, oi = (torch.from_numpy(x.array) for x in (out_b, out_v, out_i))
    res = {}
    for w in widths:
        pr = synth.banded_problem(n, p, seed + w, w, device="cuda:0")
        Mb = torch.from_numpy(pr["M_band"]).to(dev)
        XL, Y = torch.from_numpy(pr["XL"]).to(dev), torch.from_numpy(pr["Y"]).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = binding.GwasContext(Mb, XL, Y, x_dtype=x_dtype, band=w)
        torch.cuda.synchronize()
        init_s = time.perf_counter() - t0
        ctx.stream_block_async(X[0], (ob[:step], ov[:step], oi[:step]))     # warm-up
        ctx.wait()
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for s in range(steps):
            sl = slice(s * step, (s + 1) * step)
            ctx.stream_block_async(X[s], (ob[sl], ov[sl], oi[sl]))
        ctx.wait()
        el = time.perf_counter() - t0
        launches, kms, kcols = ctx.kernel_time()
        n_pad = ctx.query()["n_pad"]
        ctx.close()
        W = -(-w // 256) * 256
        # the library's choice of kernel for int8 dosages (GWAS_BAND_STEP=1
        # forces the launch per block row)
        walk = x_dtype == "i8" and W <= 512 and int(os.environ.get("GWAS_BAND_STEP", "0") or 0) == 0
        alg = 2.0 * n * w * kcols / (kms * 1e-3) / 1e12
        exe = float(n_pad) * (3.125 * W if walk else 3 * W + 128) * kcols / (kms * 1e-3) / 1e12
        rate = steps * step / el
        res[str(w)] = {"snps_per_s": rate, "init_s": init_s, "block_order": W, "n_pad": n_pad,
                       "product_ms_per_sub_block": kms / max(launches, 1),
                       "roofline": {"bound": "mfma", "achieved": alg, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                                    "frac": alg / PEAK_TFLOPS["fp64"],
                                    "work": "algorithmic 2 n w flops per SNP"},
                       "executed_tflops": exe, "executed_frac": exe / PEAK_TFLOPS["fp64"],
                       "kernel": "one launch per sub-block" if walk else "one launch per block row",
                       "rank_flags": int((oi.numpy()[:steps * step] != 0).sum())}
        log(f"[banded w={w}{'' if x_dtype == 'i8' else ' f64'}] init {init_s:.2f} s, {rate:.1f} SNP/s; product {alg:.2f} TFLOP/s algorithmic "
            f"(2nw), {exe:.2f} executed ({exe / PEAK_TFLOPS['fp64']:.3f} of peak)")
        del Mb, XL, Y, pr
        torch.cuda.empty_cache()
    for x in (out_b, out_v, out_i, blocks):
        x.close()
    xname = "int8" if x_dtype == "i8" else "float64"
    return {"n": n, "p": p, "m_per_w": steps * step, "x_dtype": xname, "precision": "fp64",
            "inputs": f"{xname} dosages in pinned host memory, queued blocks", "by_half_bandwidth": res}


def run_main(args):
    import torch
    from paper_1304_2272_amd import binding, synth
    binding.load()
    w = dict(WORKLOADS[args.workload])
    if args.step_snps:
        w["step"] = args.step_snps
    if args.x_dtype:
        w["x_dtype"] = args.x_dtype
    n, p, step = w["n"], w["p"], w["step"]
    dev = torch.device("cuda:0")
    legs = [x for x in args.legs.split(",") if x]
    if legs[0] != "fp64":
        raise SystemExit("the first leg is the float64 path, which every other leg is compared with")

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
    xdt = torch.int8 if w["x_dtype"] == "i8" else torch.float64
    nb = min(args.steps, args.host_blocks)
    blocks = host_blocks(n, args.seed, step, nb, xdt, dev)
    torch.cuda.synchronize()
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s ({nb} distinct pinned host blocks of {step} SNPs)")

    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.bitwise_not(src, out=dst)      # one element-wise kernel: reads and writes nbytes
        torch.cuda.synchronize()
        log(f"copy probe: {nbytes} bytes read and written")
        del src, dst

    res, outs = {}, {}
    for leg in legs:
        res[leg], outs[leg] = stream_leg(leg, prob_dev, blocks, args.steps, w, p)
    errs = {}
    bref, vref, iref = (o.array for o in outs["fp64"])
    for leg in legs[1:]:
        b, v, i = (o.array for o in outs[leg])
        errs[leg] = snp_errors(b, v, i, bref, vref, iref)
        log(f"[{leg}] vs fp64 over {errs[leg]['snps']} SNPs: normwise {errs[leg]['normwise_max']:.3e}, "
            f"SNP coefficient {errs[leg]['snp_se_units_max']:.3e} SE units / rel max {errs[leg]['snp_rel_max']:.3e} "
            f"median {errs[leg]['snp_rel_median']:.3e}, var {errs[leg]['var_rel_max']:.3e}")
    for o in outs.values():
        for x in o:
            x.close()
    blocks.close()
    del outs, prob_dev, prob
    torch.cuda.empty_cache()
    h2d_peak = pinned_h2d_peak()

    others = {}
    pick = set(x for x in args.other_workloads.split(",") if x)
    if not args.no_other_workloads and args.workload == "n50000_p8":
        if "n1000_p4" in pick:
            others["n1000_p4"] = compact_c1(args.seed + 1)
        if "n20000_p4" in pick:
            others["n20000_p4"] = compact_c2(args.seed + 2, args.c2_blocks)
        if "cohorts8_t64" in pick:
            others["cohorts8_t64"] = compact_c4(args.seed + 3, args.c4_steps)
        if "n10000_p4_grad" in pick:
            others["n10000_p4_grad"] = compact_c5(args.seed + 4)
        if "banded_n50000_p8" in pick:
            others["banded_n50000_p8"] = compact_banded(args.seed + 5,
                                                        [int(x) for x in args.band_widths.split(",") if x],
                                                        x_dtype=args.band_x_dtype)

    cpu = None
    if not args.no_cpu_baseline:
        cn = min(args.cpu_n, n)
        log(f"cpu baseline: oracle at n_s={cn}, {args.cpu_snps} SNPs, one pinned core ...")
        cpu = cpu_baseline(w, args.seed, cn, args.cpu_snps)
        log(f"cpu baseline {cpu['value']:.3f} SNP/s (scaled), extrapolated end to end "
            f"{cpu['extrapolated_end_to_end_s']:.0f} s")

    r = res["fp64"]
    traffic, traffic_note = measured_traffic("fp64", args.workload)
    if w["x_dtype"] != WORKLOADS[args.workload]["x_dtype"]:
        traffic, traffic_note = None, "no counter record for this dosage type"
    m = r["snps"]
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "p": p, "m": m, "snps_per_step": step,
                   "x_dtype": "int8" if w["x_dtype"] == "i8" else "f64", "precision": "fp64",
                   "inputs": (f"dosages in pinned host memory ({nb} distinct blocks of {step} SNPs), queued "
                              f"with gwas_stream_block_async and waited for with gwas_stream_wait; b, var, "
                              f"info to pinned host memory" + ("; M, X_L and y handed over in host memory"
                                                               if w.get("m_host") else "")),
                   "parallelism": "single GPU"},
        "roofline": dict(r["roofline"], traffic=traffic, traffic_note=traffic_note),
        "cpu_baseline": cpu,
        "init_s": {k: v["init_s"] for k, v in res.items()},
        "legs": {k: {kk: vv for kk, vv in v.items() if kk != "init_s"} for k, v in res.items()},
        "err_vs_fp64": errs,
        "pinned_h2d_peak_GBps": h2d_peak,
        "end_to_end_snps_per_s": m / (r["init_s"] + r["elapsed_s"]),
        "other_workloads": others,
    }
    print(json.dumps(line), flush=True)


def main():
    global SLICES
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1, help="untimed blocks per leg (one)")
    ap.add_argument("--workload", default="n50000_p8", choices=sorted(WORKLOADS))
    ap.add_argument("--legs", default="fp64,fp32,int8,bf16x3,bf16")
    ap.add_argument("--host-blocks", type=int, default=20, help="distinct pinned host blocks (cycled)")
    ap.add_argument("--step-snps", type=int, default=0)
    ap.add_argument("--x-dtype", choices=["i8", "f64"], default=None,
                    help="dosage type of the main legs (default: the workload's)")
    ap.add_argument("--seed", type=int, default=1306)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-workloads", action="store_true")
    ap.add_argument("--other-workloads", default="n1000_p4,n20000_p4,cohorts8_t64,n10000_p4_grad,banded_n50000_p8",
                    help="which compact workloads follow the main one")
    ap.add_argument("--c2-blocks", type=int, default=20)
    ap.add_argument("--c4-steps", type=int, default=2)
    ap.add_argument("--band-widths", default="256,1024,4096", help="half-bandwidths of the banded-M leg")
    ap.add_argument("--band-x-dtype", choices=["i8", "f64"], default="i8", help="dosage type of the banded-M leg")
    ap.add_argument("--slices", type=int, default=SLICES, help="int8 digits per entry of L^-1 in the int8 leg (4..6)")
    ap.add_argument("--cpu-n", type=int, default=4096)
    ap.add_argument("--cpu-snps", type=int, default=512)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    SLICES = args.slices

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    run_main(args)


if __name__ == "__main__":
    main()
