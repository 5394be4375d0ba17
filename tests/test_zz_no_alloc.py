"""gwas_stream_block_noalloc, the entry point for callers that cannot
allocate: its sub-blocks keep their per-SNP scratch in the library's static
device buffer.  Its outputs must equal gwas_stream_block's on the same
context bit for bit (a SNP's arithmetic does not depend on the sub-block it
arrives in), over two calls in a row whose second is smaller, in every
precision mode; and it must refuse host memory and sizes whose scratch does
not fit the buffer."""

import numpy as np
import pytest

from paper_1304_2272_amd import binding, synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _outs(m, t, p, dev):
    import torch
    return (torch.full((m, t, p), float("nan"), dtype=torch.float64, device=dev),
            torch.full((m,), float("nan"), dtype=torch.float64, device=dev),
            torch.full((m,), -7, dtype=torch.int32, device=dev))


@pytest.mark.parametrize("precision,x_dtype,dev_block,n,p,t", [
    ("fp64", "f64", 512, 1500, 4, 1),      # three noalloc sub-blocks, ragged tail
    ("fp64", "i8", 0, 2300, 8, 3),         # traits: p + t cross terms
    ("fp32", "i8", 384, 700, 3, 1),
    ("int8", "i8", 256, 3000, 5, 2),
    ("bf16", "f64", 0, 900, 2, 1),
    ("bf16x3", "f64", 640, 1000, 4, 1),
])
def test_noalloc_equals_stream_block(precision, x_dtype, dev_block, n, p, t):
    import torch
    dev = torch.device("cuda:0")
    seed = 4100 + n
    prob = synth.make_problem(n, p, seed, t=t)
    xdt = np.int8 if x_dtype == "i8" else np.float64
    with binding.GwasContext(prob["M"], prob["XL"], prob["Y"], precision=precision, x_dtype=x_dtype,
                             dev_block=dev_block, slices=6 if precision == "int8" else 0) as ctx:
        for call, m in enumerate((1337, 300)):        # the second call is smaller
            _say(f"{precision}/{x_dtype} n={n} p={p} t={t} dev_block={dev_block}: call {call}, {m} SNPs")
            # column stride a multiple of 16 bytes (the call reads in place)
            ld = -(-n * np.dtype(xdt).itemsize // 16) * 16 // np.dtype(xdt).itemsize
            Xpad = torch.zeros((m, ld), dtype=torch.int8 if x_dtype == "i8" else torch.float64, device=dev)
            Xpad[:, :n] = torch.from_numpy(synth.snp_block(n, seed, 2000 * call, m, dtype=xdt)).to(dev)
            X = Xpad[:, :n]
            ref = ctx.stream_block(X)
            got = _outs(m, t, p, dev)
            ctx.stream_block_noalloc(X, got)
            torch.cuda.synchronize()
            for r, g in zip(ref, got):
                assert torch.equal(r.view(-1).view(torch.int64) if r.dtype == torch.float64 else r,
                                   g.view(-1).view(torch.int64) if g.dtype == torch.float64 else g)
            assert bool((got[2] == 0).all())


def test_noalloc_without_var_info_and_then_blocking_calls():
    # optional outputs left out; a blocking call after a queued noalloc call
    # on the same context sees a consistent context
    import torch
    dev = torch.device("cuda:0")
    n, p, m, seed = 1100, 4, 900, 4201
    prob = synth.make_problem(n, p, seed)
    X = torch.from_numpy(synth.snp_block(n, seed, 0, m)).to(dev)
    with binding.GwasContext(prob["M"], prob["XL"], prob["Y"], dev_block=256) as ctx:
        b, _, _ = _outs(m, 1, p, dev)
        ctx.stream_block_noalloc(X, (b, None, None))
        ref = ctx.stream_block(X)
        torch.cuda.synchronize()
        assert torch.equal(b.view(torch.int64), ref[0].view(torch.int64))


def test_noalloc_refuses_host_memory_and_oversized_scratch():
    import torch
    dev = torch.device("cuda:0")
    n, p, m, seed = 600, 3, 64, 4202
    prob = synth.make_problem(n, p, seed)
    X = synth.snp_block(n, seed, 0, m)
    with binding.GwasContext(prob["M"], prob["XL"], prob["Y"]) as ctx:
        L = binding.load()
        b = np.empty((m, 1, p))
        Xd = torch.from_numpy(X).to(dev)
        bd = torch.empty((m, 1, p), dtype=torch.float64, device=dev)
        # host dosages, then host outputs: refused, nothing queued
        assert L.gwas_stream_block_noalloc(ctx._h, X.ctypes.data, n, m, bd.data_ptr(), p, None, None) == 1
        assert L.gwas_stream_block_noalloc(ctx._h, Xd.data_ptr(), n, m, b.ctypes.data, p, None, None) == 1
        assert "device memory" in L.gwas_last_error(ctx._h).decode()
        # the context stays usable
        ctx.stream_block(Xd)
    # 128 SNP columns of float64 partial sums at n_pad = 32,768 with
    # p + t = 276 cross terms need 2.3 GB of scratch: refused
    n, p, t = 32_768, 20, 256
    _say(f"n={n} p={p} t={t}: scratch larger than the static buffer")
    M = torch.eye(n, dtype=torch.float64, device=dev)
    XL = torch.randn(n, p - 1, dtype=torch.float64, device=dev)
    Y = torch.randn(n, t, dtype=torch.float64, device=dev)
    with binding.GwasContext(M, XL, Y, dev_block=128) as ctx:
        del M
        Xd = torch.zeros((4, n), dtype=torch.float64, device=dev)
        with pytest.raises(binding.GwasError) as ei:
            ctx.stream_block_noalloc(Xd, _outs(4, t, p, dev))
        assert ei.value.code == 1 and "static buffer" in str(ei.value)
