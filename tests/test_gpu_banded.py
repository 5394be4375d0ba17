"""Banded M (the variant of Section 5.1: relatives grouped near the
diagonal): the block-bidiagonal factor and the block forward substitution of
each streamed block against the CPU oracle, which takes the same M dense."""

import numpy as np
import pytest

from oracle import GLSOracle
from paper_1304_2272_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(*a):
    print(*a, flush=True)


def normwise(b, bref):
    num = np.linalg.norm((b - bref).reshape(b.shape[0], -1), axis=1)
    den = np.linalg.norm(bref.reshape(b.shape[0], -1), axis=1)
    return float(np.max(num / den))


@pytest.mark.parametrize("n,w,p,t,m,x_dtype,dev_block", [
    (3000, 100, 4, 1, 1500, "f64", 0),      # W = 256, 12 block rows, n not a multiple of W
    (2100, 300, 8, 1, 1300, "i8", 256),     # W = 512, ragged sub-blocks
    (700, 650, 3, 2, 400, "f64", 128),      # one block row (W = 768 >= n), two traits
    (5000, 1000, 3, 1, 900, "i8", 0),       # W = 1024, 5 block rows
    (1290, 256, 5, 1, 333, "f64", 128),     # w = W exactly
    (1800, 400, 4, 3, 500, "i8", 0),        # W = 512 in one launch, three traits
    (6000, 1500, 4, 1, 700, "i8", 0),       # W = 1,536: one launch per block row, loaded straight into LDS
    (4000, 1300, 3, 2, 300, "i8", 128),     # W = 1,536, ragged last block row, two traits
])
def test_banded_vs_oracle(n, w, p, t, m, x_dtype, dev_block):
    seed = 5100 + n + w
    _say(f"banded n={n} w={w} p={p} t={t} m={m} {x_dtype} dev_block={dev_block}")
    prob = synth.banded_problem(n, p, seed, w, t=t)
    xdt = np.int8 if x_dtype == "i8" else np.float64
    XR = synth.snp_block(n, seed, 0, m, dtype=xdt)
    with binding.GwasContext(prob["M_band"], prob["XL"], prob["Y"], x_dtype=x_dtype, dev_block=dev_block,
                             band=w) as ctx:
        b, var, info = ctx.stream_block(XR)
    M = synth.band_to_dense(prob["M_band"])
    bo, vo, io = GLSOracle(M, prob["XL"], prob["Y"]).solve(XR)
    err = normwise(b, bo)
    verr = float(np.max(np.abs(var - vo) / vo))
    _say(f"  normwise {err:.3e}, var {verr:.3e}")
    assert np.array_equal(info, io) and (io == 0).all()
    assert err < TOL and verr < TOL


def test_banded_equals_dense_path_and_partitions():
    # the same M through the dense path; and a SNP's result does not depend
    # on the block or sub-block it comes in (bit for bit)
    import torch
    n, w, p, m, seed = 1800, 200, 4, 1000, 5201
    prob = synth.banded_problem(n, p, seed, w)
    M = synth.band_to_dense(prob["M_band"])
    XR = synth.snp_block(n, seed, 0, m)
    with binding.GwasContext(M, prob["XL"], prob["Y"]) as ctx:
        bd, vd, _ = ctx.stream_block(XR)
    dev = torch.device("cuda:0")
    Mb = torch.from_numpy(prob["M_band"]).to(dev)
    XL, Y = torch.from_numpy(prob["XL"]).to(dev), torch.from_numpy(prob["Y"]).to(dev)
    with binding.GwasContext(Mb, XL, Y, band=w, dev_block=256) as ctx:
        Xd = torch.from_numpy(XR).to(dev)
        b1, v1, _ = ctx.stream_block(Xd)
        parts = [ctx.stream_block(Xd[a:z]) for a, z in ((0, 129), (129, 700), (700, m))]
    b1, v1 = b1.cpu().numpy(), v1.cpu().numpy()
    err = normwise(b1, bd)
    _say(f"banded vs dense path: normwise {err:.3e}")
    assert err < 1e-12 and float(np.max(np.abs(v1 - vd) / vd)) < 1e-12
    b2 = np.concatenate([q[0].cpu().numpy() for q in parts])
    assert np.array_equal(b2, b1)


def test_banded_not_spd_and_rank_deficient_snp():
    n, w, p, seed = 900, 120, 4, 5301
    prob = synth.banded_problem(n, p, seed, w)
    XR = synth.snp_block(n, seed, 0, 50)
    XR[7] = 1.0                                   # collinear with the intercept
    with binding.GwasContext(prob["M_band"], prob["XL"], prob["Y"], band=w) as ctx:
        b, var, info = ctx.stream_block(XR)
    assert info[7] == p and np.isnan(b[7]).all()
    assert (np.delete(info, 7) == 0).all()
    bad = prob["M_band"].copy()
    bad[613, 0] = -1.0                            # M(613, 613) < 0: leading minor 614 fails
    with pytest.raises(binding.GwasError) as ei:
        binding.GwasContext(bad, prob["XL"], prob["Y"], band=w)
    assert ei.value.code == 2 and ei.value.info == 614


def test_banded_calls_that_need_the_dense_factor_are_refused():
    import torch
    n, w, p, seed = 600, 60, 3, 5401
    prob = synth.banded_problem(n, p, seed, w)
    XR = synth.snp_block(n, seed, 0, 40)
    with binding.GwasContext(prob["M_band"], prob["XL"], prob["Y"], band=w) as ctx:
        for call in (lambda: ctx.backward_begin(), lambda: ctx.autotune(XR),
                     lambda: binding.stream_group([ctx], [XR])):
            with pytest.raises(binding.GwasError) as ei:
                call()
            assert ei.value.code == 1
        b, _, info = ctx.stream_block(XR)        # the context stays usable
        assert (info == 0).all()


@pytest.mark.parametrize("n,w,p,m", [
    (3000, 200, 5, 9000),      # W = 256, 12 block rows; 32 columns per workgroup, ragged last workgroup
    (2600, 400, 4, 9000),      # W = 512, 6 block rows (the last one partly past n)
    (1100, 256, 3, 700),       # W = 256, 5 block rows; 16 columns per workgroup
    (1500, 450, 3, 600),       # W = 512, 3 block rows; 16 columns per workgroup
])
def test_banded_one_launch_equals_block_row_launches(n, w, p, m, monkeypatch):
    # int8 dosages with W of 256 or 512 run every block row of a sub-block in
    # one launch, Z kept on chip; the launch per block row (GWAS_BAND_STEP=1)
    # gives the same bits, a SNP's result does not depend on the call it
    # comes in, and a sample of SNPs agrees with the oracle on the dense M
    seed = 5500 + n + w
    _say(f"banded one launch n={n} w={w} p={p} m={m}")
    prob = synth.banded_problem(n, p, seed, w)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    monkeypatch.delenv("GWAS_BAND_STEP", raising=False)
    with binding.GwasContext(prob["M_band"], prob["XL"], prob["Y"], x_dtype="i8", band=w) as ctx:
        b1, v1, i1 = ctx.stream_block(XR)
        cut = m - 513 if m > 8192 else m // 3
        parts = [ctx.stream_block(XR[:cut]), ctx.stream_block(XR[cut:])]
    monkeypatch.setenv("GWAS_BAND_STEP", "1")
    with binding.GwasContext(prob["M_band"], prob["XL"], prob["Y"], x_dtype="i8", band=w) as ctx:
        b2, v2, i2 = ctx.stream_block(XR)
    assert (i1 == 0).all() and np.array_equal(i1, i2)
    assert np.array_equal(b1, b2) and np.array_equal(v1, v2)
    assert np.array_equal(np.concatenate([q[0] for q in parts]), b1)
    assert np.array_equal(np.concatenate([q[1] for q in parts]), v1)
    rng = np.random.default_rng(seed)
    pick = np.unique(np.concatenate([[0, 31, 32, m - 1], rng.choice(m, 60, replace=False)]))
    bo, vo, io = GLSOracle(synth.band_to_dense(prob["M_band"]), prob["XL"], prob["Y"]).solve(XR[pick])
    err = normwise(b1[pick], bo)
    verr = float(np.max(np.abs(v1[pick] - vo) / vo))
    _say(f"  bit-equal to the per-block-row launches; oracle sample normwise {err:.3e}, var {verr:.3e}")
    assert err < TOL and verr < TOL


@pytest.mark.parametrize("n,w,p,m", [
    (1291, 200, 4, 700),       # W = 256, n odd: the last stage ends one K into a 16-byte piece
    (2999, 700, 3, 500),       # W = 768, 4 block rows, the last one mostly past n
])
def test_banded_float64_dosages_strided_nan_padding(n, w, p, m):
    # float64 dosages in device memory with a stride past n whose padding
    # holds NaN: every K at or past n is read as zero, so the padding (and
    # the next column's first values) never reach b or var
    import torch
    seed = 5600 + n + w
    _say(f"banded float64 strided dosages n={n} w={w} p={p} m={m}")
    prob = synth.banded_problem(n, p, seed, w)
    XR = synth.snp_block(n, seed, 0, m)
    ld = n + 7 if n % 2 else n + 6
    dev = torch.device("cuda:0")
    Xp = torch.full((m, ld), float("nan"), dtype=torch.float64, device=dev)
    Xp[:, :n] = torch.from_numpy(XR).to(dev)
    with binding.GwasContext(prob["M_band"], prob["XL"], prob["Y"], band=w) as ctx:
        b, var, info = ctx.stream_block(Xp[:, :n])
        bh, vh, _ = ctx.stream_block(XR)
    b, var, info = b.cpu().numpy(), var.cpu().numpy(), info.cpu().numpy()
    bo, vo, io = GLSOracle(synth.band_to_dense(prob["M_band"]), prob["XL"], prob["Y"]).solve(XR)
    err = normwise(b, bo)
    verr = float(np.max(np.abs(var - vo) / vo))
    _say(f"  normwise {err:.3e}, var {verr:.3e}")
    assert np.array_equal(info, io) and (io == 0).all()
    assert err < TOL and verr < TOL
    assert np.array_equal(b, bh) and np.array_equal(var, vh)
