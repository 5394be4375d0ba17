"""GPU parity: the HIP library through its C ABI against the CPU oracle, on
seeded inputs that span several tiles, ragged sub-blocks and edge cases."""

import numpy as np
import pytest

from oracle import GLSOracle
from paper_1304_2272_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10   # max_i ||b_i - b_i^ref|| / ||b_i^ref||
TOL_FP32 = 1e-8


def _say(*a):
    print(*a, flush=True)


def torch_equal(x, y):
    return bool(np.array_equal(np.asarray(x), np.asarray(y)))


def normwise(b, bref):
    num = np.linalg.norm((b - bref).reshape(b.shape[0], -1), axis=1)
    den = np.linalg.norm(bref.reshape(b.shape[0], -1), axis=1)
    return float(np.max(num / den)) if b.shape[0] else 0.0


U32, U16 = 2.0 ** -24, 2.0 ** -8   # unit roundoff of float32 and bfloat16


def snp_errors(b, bref, var, vref, ok):
    """(max relative error of the SNP coefficient, of var, and the SNP
    coefficient's error in standard-error units) over the SNPs in ok."""
    if not ok.any():
        return 0.0, 0.0, 0.0
    bs, brs = b[ok][..., -1], bref[ok][..., -1]
    d = np.abs(bs - brs)
    sd = np.sqrt(vref[ok])
    rel = float(np.max(d / np.abs(brs)))
    vrel = float(np.max(np.abs(var[ok] - vref[ok]) / vref[ok]))
    se = float(np.max(d / (sd[:, None] if d.ndim == 2 else sd)))
    return rel, vrel, se


def reduced_floor(orc, XR, b, bref, var, vref, ok, u):
    """The stated floor of the reduced-precision modes: S_BR is their only
    reduced-precision quantity and c_i is float64-exact, so b_SNP = c_i / s_i
    and var_i = 1 / s_i carry the relative error of s_i, at most
    16 u kappa_i with kappa_i = S_BR / s_i = (x^T M^-1 x) var_i.  Returns the
    worst ratio of error to that limit over b_SNP and var, and max kappa."""
    if not ok.any():
        return 0.0, 0.0
    N, _ = orc.normal_equations(XR[ok])
    kappa = N[:, -1, -1] * vref[ok]
    lim = 16.0 * u * kappa
    rel = np.abs(b[ok][..., -1] - bref[ok][..., -1]) / np.abs(bref[ok][..., -1])
    vrel = np.abs(var[ok] - vref[ok]) / vref[ok]
    worst = max(float(np.max(rel / (lim[:, None] if rel.ndim == 2 else lim))), float(np.max(vrel / lim)))
    return worst, float(kappa.max())


def run(prob, XR, **kw):
    with binding.GwasContext(prob["M"], prob["XL"], prob["Y"], **kw) as ctx:
        return ctx.stream_block(XR)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    binding.load()


def test_fp64_n1000_p4_all_snps():
    n, p, m, seed = 1000, 4, 10_000, 1304
    _say(f"fp64 n={n} p={p} m={m} seed={seed}")
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m)
    b, var, info = run(prob, XR)
    bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    assert np.array_equal(info, io)
    err = normwise(b, bo)
    verr = float(np.max(np.abs(var - vo) / vo))
    _say(f"  max normwise err {err:.3e}, var err {verr:.3e}")
    assert err < TOL_FP64 and verr < TOL_FP64


@pytest.mark.parametrize("x_dtype", ["f64", "i8"])
@pytest.mark.parametrize("n,p,m,dev_block", [(777, 3, 1500, 256), (130, 5, 300, 128),
                                               (4, 4, 37, 128), (2, 2, 41, 128), (1283, 20, 400, 384)])
def test_ragged_shapes(x_dtype, n, p, m, dev_block):
    # n = p: X_i is square, singular when its dosage column is a multiple of
    # the intercept (n = p = 2: equal dosages), which both sides must flag
    seed = 7 + n
    _say(f"ragged x={x_dtype} n={n} p={p} m={m} dev_block={dev_block}")
    prob = synth.make_problem(n, p, seed, k=max(50, n // 2))
    dt = np.int8 if x_dtype == "i8" else np.float64
    XR = synth.snp_block(n, seed, 0, m, dtype=dt)
    b, var, info = run(prob, XR, x_dtype=x_dtype, dev_block=dev_block)
    bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    ok = io == 0
    assert np.array_equal(info, io)
    err = normwise(b[ok], bo[ok])
    _say(f"  err {err:.3e}")
    assert err < TOL_FP64


@pytest.mark.parametrize("n,p,m,dev_block", [(777, 3, 1500, 256), (130, 5, 300, 128),
                                               (4, 4, 37, 128), (2, 2, 41, 128), (1283, 20, 400, 384),
                                               (2049, 4, 531, 512)])
def test_ragged_shapes_int8_slices(n, p, m, dev_block):
    # interior stages stream straight to LDS; the last column tile of a
    # sub-block and the stages crossing n take the zero-filled edge path
    seed = 17 + n
    _say(f"ragged int8 slices n={n} p={p} m={m} dev_block={dev_block}")
    prob = synth.make_problem(n, p, seed, k=max(50, n // 2))
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    b, var, info = run(prob, XR, precision="int8", x_dtype="i8", dev_block=dev_block)
    bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    ok = io == 0
    assert np.array_equal(info, io)
    err = normwise(b[ok], bo[ok])
    _say(f"  err {err:.3e}")
    # tiny n (n = p) cancels most of S_BR in s = S_BR - u^T u, which
    # magnifies the slices' 1e-14 truncation; a misplaced chunk or row
    # would be off by O(1).  The mixed-precision bar applies here; the
    # float64-level check of the slices is test_int8_slices.
    assert err < 1e-8


def test_partition_independence_and_device_io():
    import torch
    n, p, m, seed = 900, 4, 2000, 31
    _say(f"partition n={n} p={p} m={m}")
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m)
    b1, v1, i1 = run(prob, XR, dev_block=128)
    b2, v2, i2 = run(prob, XR, dev_block=1024)
    assert np.array_equal(b1, b2) and np.array_equal(v1, v2)
    # one call per SNP range gives the same bits
    with binding.GwasContext(prob["M"], prob["XL"], prob["Y"], dev_block=512) as ctx:
        parts = [ctx.stream_block(XR[a:b_])[0] for a, b_ in [(0, 1), (1, 700), (700, 2000)]]
    assert np.array_equal(np.concatenate(parts), b1)
    # device-resident inputs and outputs
    dev = torch.device("cuda:0")
    Md = torch.from_numpy(prob["M"]).to(dev)
    XLd = torch.from_numpy(prob["XL"]).to(dev)
    Yd = torch.from_numpy(prob["Y"]).to(dev)
    XRd = torch.from_numpy(XR).to(dev)
    with binding.GwasContext(Md, XLd, Yd, dev_block=128) as ctx:
        bd, vd, idd = ctx.stream_block(XRd)
        torch.cuda.synchronize()
    assert np.array_equal(bd.cpu().numpy(), b1)
    assert np.array_equal(vd.cpu().numpy(), v1)


@pytest.mark.parametrize("precision,x_dtype", [("fp64", "i8"), ("fp64", "f64"), ("fp32", "i8"), ("bf16", "i8"),
                                               ("int8", "i8"), ("fp32", "f64")])
def test_strided_device_dosages_ignore_padding(precision, x_dtype):
    # dosages read straight from a device array whose columns are ldx > n
    # apart, with garbage between element n-1 and the next column: the
    # products load whole 16-byte chunks and clear (or range-check) what lies
    # past n, so the result equals the compact input bit for bit
    import torch
    n, p, m, seed = 777, 4, 700, 41
    _say(f"strided {precision} x={x_dtype} n={n} m={m}")
    prob = synth.make_problem(n, p, seed)
    dt = np.int8 if x_dtype == "i8" else np.float64
    XR = synth.snp_block(n, seed, 0, m, dtype=dt)
    dev = torch.device("cuda:0")
    ldx = (n + 15) // 16 * 16 + 32
    big = torch.full((m, ldx), 99 if x_dtype == "i8" else 1e300, dtype=torch.from_numpy(XR).dtype, device=dev)
    big[:, :n] = torch.from_numpy(XR).to(dev)
    strided = big[:, :n]
    assert strided.stride(0) == ldx
    kw = dict(precision=precision, x_dtype=x_dtype, dev_block=256)
    b0, v0, i0 = run(prob, torch.from_numpy(XR).to(dev).contiguous(), **kw)
    b1, v1, i1 = run(prob, strided, **kw)
    torch.cuda.synchronize()
    assert torch_equal(i0.cpu(), i1.cpu())
    assert torch_equal(b0.cpu(), b1.cpu()) and torch_equal(v0.cpu(), v1.cpu())


def test_traits_and_max_p():
    n, p, t, m, seed = 600, 20, 5, 700, 44
    _say(f"traits n={n} p={p} t={t} m={m}")
    prob = synth.make_problem(n, p, seed, t=t)
    XR = synth.snp_block(n, seed, 0, m)
    b, var, info = run(prob, XR)
    bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    assert b.shape == (m, t, p)
    err = normwise(b, bo)
    _say(f"  err {err:.3e}")
    assert err < TOL_FP64


def test_planted_coefficients():
    n, p, m, seed = 2000, 6, 1024, 5
    _say(f"planted n={n} p={p} m={m}")
    prob = synth.make_problem(n, p, seed, noise=False)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    b, _, info = run(prob, XR, x_dtype="i8")
    want = np.concatenate([prob["beta"][:, 0], [0.0]])
    assert (info == 0).all()
    assert np.max(np.abs(b[:, 0, :] - want)) < 1e-9


def test_rank_deficient_snp_and_not_spd():
    n, p, m, seed = 300, 4, 64, 9
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m)
    XR[5] = 2.0
    XR[60] = 0.0
    b, var, info = run(prob, XR)
    _, _, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    assert list(np.flatnonzero(info)) == [5, 60] and list(np.flatnonzero(io)) == [5, 60]
    assert np.isnan(b[5]).all() and np.isnan(var[60])
    # M with a negative leading minor of order 101
    M = prob["M"].copy()
    M[100, 100] = -1.0
    with pytest.raises(binding.GwasError) as ei:
        binding.GwasContext(M, prob["XL"], prob["Y"])
    assert ei.value.code == 2 and ei.value.info == 101
    # a rank-deficient X_L
    XL = prob["XL"].copy()
    XL[:, 2] = XL[:, 0]
    with pytest.raises(binding.GwasError) as ei:
        binding.GwasContext(prob["M"], XL, prob["Y"])
    assert ei.value.code == 3


RANK_TOL = {"fp64": 1e-10, "int8": 1e-10, "fp32": 1e-6, "bf16x3": 1e-6, "bf16": 1e-2}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "bf16"])
def test_rank_flag_is_whitened_r2_above_one_minus_tol(precision):
    # info = p exactly when s_i <= tol S_BR, i.e. when the whitened R^2 of
    # x_i on X_L is at least 1 - tol: collinear SNPs in every mode and, in
    # the reduced modes, SNPs too close to collinear for their product to
    # resolve s_i (b and var NaN).  SNPs are planted at 1 - R^2 from 0.5
    # down to 1e-12 and at exact collinearity; those within a factor 4 of
    # the tolerance may go either way.
    n, p, seed = 600, 4, 303
    prob = synth.make_problem(n, p, seed)
    M, XL = prob["M"], prob["XL"]
    Li = np.linalg.inv(np.linalg.cholesky(M))
    A = Li @ XL
    Qa, _ = np.linalg.qr(A)
    rng = np.random.default_rng(seed)
    gaps = np.array([0.5, 0.1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10, 1e-11, 1e-12, 0.0])
    XR = np.empty((len(gaps) * 3, n))
    target = np.empty(len(XR))
    for k in range(len(XR)):
        gap = gaps[k % len(gaps)]
        u = Qa @ rng.standard_normal(Qa.shape[1])        # in the span of the whitened covariates
        v = rng.standard_normal(n)
        v -= Qa @ (Qa.T @ v)                             # orthogonal to it
        zw = u / np.linalg.norm(u) * np.sqrt(1.0 - gap) + v / np.linalg.norm(v) * np.sqrt(gap)
        XR[k] = np.linalg.solve(Li, zw)                  # x = L zw, so L^-1 x = zw
        zx = Li @ XR[k]
        target[k] = 1.0 - np.sum((Qa.T @ zx) ** 2) / np.sum(zx ** 2)
    # the planted SNPs with an exact zero gap are exact combinations of X_L
    exact = gaps[np.arange(len(XR)) % len(gaps)] == 0.0
    XR[exact] = (XL @ rng.standard_normal((p - 1, int(exact.sum())))).T
    target[exact] = 0.0
    tol = RANK_TOL[precision]
    _say(f"rank flag {precision}: tol {tol:g}, gaps {gaps[0]:g}..{gaps[-2]:g} and 0")
    b, var, info = run(prob, XR, precision=precision)
    flagged = info != 0
    sure_in = target <= tol / 4
    sure_out = target >= 4 * tol
    _say(f"  flagged {int(flagged.sum())} of {len(XR)}; must {int(sure_in.sum())}, must not {int(sure_out.sum())}")
    assert np.all(flagged[sure_in]) and not np.any(flagged[sure_out])
    assert np.all(info[flagged] == p) and np.all(np.isnan(b[flagged])) and np.all(np.isnan(var[flagged]))
    assert np.all(np.isfinite(b[~flagged])) and np.all(np.isfinite(var[~flagged]))
    if precision == "fp64":
        # the oracle takes the same decision outside the band around tol
        # (a SNP planted at 1 - R^2 = tol goes either way on either side)
        _, _, io = GLSOracle(M, XL, prob["Y"]).solve(XR)
        clear = sure_in | sure_out
        assert np.array_equal(info[clear], io[clear])


@pytest.mark.parametrize("precision,tol", [("fp32", TOL_FP32), ("bf16", 1e-2), ("int8", TOL_FP64)])
def test_reduced_precision_vs_oracle(precision, tol):
    n, p, m, seed = 1500, 8, 3000, 77
    _say(f"{precision} n={n} p={p} m={m}")
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    b, var, info = run(prob, XR, precision=precision, x_dtype="i8")
    bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    err = normwise(b, bo)
    _say(f"  normwise err {err:.3e}")
    assert np.array_equal(info, io)
    assert err < tol


TILE_SHAPES = {"fp64": [0, 1, 2, 3, 4, 5, 7], "fp32": [1, 2, 3, 5, 6], "bf16": [1, 2, 3, 5, 6], "int8": [0, 1, 2, 3, 4, 5, 6]}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_every_tile_shape(precision, monkeypatch):
    # every tile shape the library may pick gives the oracle's answer
    n, p, m, seed = 700, 5, 900, 123
    prob = synth.make_problem(n, p, seed, k=300)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    bo, _, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    tol = {"fp64": TOL_FP64, "fp32": TOL_FP32, "bf16": 1e-2}[precision]
    ref = None
    for cfg in TILE_SHAPES[precision]:
        monkeypatch.setenv("GWAS_TRMM_CFG", str(cfg))
        _say(f"{precision} tile shape {cfg} n={n} m={m}")
        b, _, info = run(prob, XR, precision=precision, x_dtype="i8", dev_block=384)
        assert np.array_equal(info, io)
        err = normwise(b, bo)
        _say(f"  err {err:.3e}")
        assert err < tol
        if precision == "fp64":
            # float64 sums differ between shapes only in rounding order
            ref = b if ref is None else ref
            assert normwise(b, ref) < 1e-13


@pytest.mark.parametrize("n,m,dev_block", [(3000, 700, 384), (1290, 300, 128)])
def test_fp64_direct_load_float64_dosages(n, m, dev_block, monkeypatch):
    # the float64 tile loaded straight into LDS (7) with float64 dosages,
    # non-integer ones included, against the oracle; the elements past n of
    # each column (NaN here) never reach the sums, so a strided block gives
    # the bits of a packed one; the register-staged tile (3) agrees to
    # rounding
    import torch
    p, seed = 5, 812
    prob = synth.make_problem(n, p, seed, k=max(50, n // 3))
    XR = synth.snp_block(n, seed, 0, m)
    XR[::3] += np.random.default_rng(seed).uniform(-0.4, 0.4, size=XR[::3].shape)   # imputed dosages
    monkeypatch.setenv("GWAS_TRMM_CFG", "7")
    _say(f"fp64 shape 7, float64 dosages n={n} m={m} dev_block={dev_block}")
    b, var, info = run(prob, XR, precision="fp64", x_dtype="f64", dev_block=dev_block)
    dev = torch.device("cuda:0")
    big = torch.full((m, n + 48), float("nan"), dtype=torch.float64, device=dev)
    big[:, :n] = torch.from_numpy(XR).to(dev)
    bs, vs, is_ = run(prob, big[:, :n], precision="fp64", x_dtype="f64", dev_block=dev_block)
    assert np.array_equal(b, bs.cpu().numpy()) and np.array_equal(var, vs.cpu().numpy())
    bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    assert np.array_equal(info, io) and (io == 0).all()
    err = normwise(b, bo)
    _say(f"  normwise {err:.3e} against the oracle")
    assert err < TOL_FP64 and float(np.max(np.abs(var - vo) / vo)) < TOL_FP64
    monkeypatch.setenv("GWAS_TRMM_CFG", "3")
    b3, _, _ = run(prob, XR, precision="fp64", x_dtype="f64", dev_block=dev_block)
    assert normwise(b, b3) < 1e-13


def test_bf16_float64_dosages_every_tile_shape(monkeypatch):
    # float64 (imputed) dosages are rounded to bfloat16 once per sub-block
    # for the bfloat16 product; every tile shape that reads them gives the
    # oracle's answer to the bfloat16 mode's accuracy, the default among them
    n, p, m, seed = 700, 5, 900, 124
    prob = synth.make_problem(n, p, seed, k=300)
    XR = synth.imputed_block(n, seed, 0, m)
    bo, _, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    for cfg in (None, 1, 2, 5, 6):
        if cfg is None:
            monkeypatch.delenv("GWAS_TRMM_CFG", raising=False)
        else:
            monkeypatch.setenv("GWAS_TRMM_CFG", str(cfg))
        b, _, info = run(prob, XR, precision="bf16", x_dtype="f64", dev_block=384)
        err = normwise(b, bo)
        _say(f"bf16 float64 dosages, tile shape {cfg}: err {err:.3e}")
        assert np.array_equal(info, io) and err < 1e-2


def rounding_bound(prob, XR, b_ref, u_store, u_acc):
    """First-order bound of each SNP's normwise error of b when z = L^-1 x
    is formed from L^-1 rounded with unit roundoff u_store and summed with
    unit roundoff u_acc (any order), and every other quantity is exact:
    |dz_r| <= (u_store + n u_acc) (|L^-1| |x|)_r, dS_BR <= 2 sum_r |z_r| |dz_r|,
    and a change d of S_BR moves b by -d b_p S^-1 e_p."""
    M, XL = prob["M"], prob["XL"]
    n = M.shape[0]
    Li = np.linalg.inv(np.linalg.cholesky(M))
    X = XR.astype(np.float64)
    Z = Li @ X.T
    dz = (u_store + n * u_acc) * (np.abs(Li) @ np.abs(X).T)
    dS = 2.0 * np.sum(np.abs(Z) * dz, axis=0)
    Minv = np.linalg.inv(M)
    out = np.zeros(X.shape[0])
    for i in range(X.shape[0]):
        Xi = np.column_stack([XL, X[i]])
        S = Xi.T @ Minv @ Xi
        col = np.linalg.solve(S, np.eye(S.shape[0])[:, -1])
        bi = b_ref[i, 0]
        out[i] = np.linalg.norm(col) * dS[i] * abs(bi[-1]) / np.linalg.norm(bi)
    return out


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("cfg", [3, 6])
@pytest.mark.parametrize("n,p,m,dev_block", [(17, 3, 60, 128), (130, 5, 300, 128), (255, 4, 300, 256),
                                               (257, 4, 531, 512), (777, 3, 1500, 256)])
def test_reduced_precision_ragged_within_rounding_bound(precision, cfg, n, p, m, dev_block, monkeypatch):
    # n below one stage, one tile and just past a tile; ragged column tiles.
    # At small n the cancellation in S_BR - u^T S_TL^-1 u magnifies the
    # rounding of L^-1 past the 1e-8 bar of large n, so each SNP is held to
    # twice the first-order rounding bound instead; a lost or misplaced
    # chunk of the product is off by O(1).
    seed = 29 + n
    monkeypatch.setenv("GWAS_TRMM_CFG", str(cfg))
    _say(f"{precision} tile shape {cfg} n={n} p={p} m={m} dev_block={dev_block}")
    prob = synth.make_problem(n, p, seed, k=max(50, n // 2))
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    b, var, info = run(prob, XR, precision=precision, x_dtype="i8", dev_block=dev_block)
    orc = GLSOracle(prob["M"], prob["XL"], prob["Y"])
    bo, vo, io = orc.solve(XR)
    assert np.array_equal(info, io)
    ok = io == 0
    u = U32 if precision == "fp32" else U16
    bound = rounding_bound(prob, XR[ok], bo[ok], u, 2.0 ** -24)
    num = np.linalg.norm((b[ok] - bo[ok]).reshape(int(ok.sum()), -1), axis=1)
    err = num / np.linalg.norm(bo[ok].reshape(int(ok.sum()), -1), axis=1)
    worst, kmax = reduced_floor(orc, XR, b, bo, var, vo, ok, u)
    _say(f"  err {err.max():.3e}, worst err / bound {np.max(err / (bound + 1e-300)):.3f}; "
         f"SNP coefficient and var against 16 u kappa: {worst:.3f} (kappa <= {kmax:.1f})")
    assert np.all(err <= 2.0 * bound + 1e-13)
    assert worst <= 1.0


@pytest.mark.parametrize("slices,tol", [(4, 1e-8), (5, 1e-9), (6, TOL_FP64)])
def test_int8_slices(slices, tol):
    # int8 digits of L^-1 against int8 dosages, exact int32 sums
    n, p, m, seed = 2100, 6, 2500, 91
    _say(f"int8 slices={slices} n={n} p={p} m={m}")
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    b, var, info = run(prob, XR, precision="int8", x_dtype="i8", slices=slices, dev_block=1024)
    bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    err = normwise(b, bo)
    verr = float(np.max(np.abs(var - vo) / vo))
    _say(f"  normwise err {err:.3e} var err {verr:.3e}")
    assert np.array_equal(info, io)
    assert err < tol and verr < 100 * tol


@pytest.mark.parametrize("n,p,m,dev_block", [(2100, 6, 2500, 1024), (777, 3, 1500, 256), (130, 5, 300, 128),
                                               (17, 3, 60, 128), (1030, 4, 333, 384)])
@pytest.mark.parametrize("slices", [4, 5, 6])
def test_int8_slice_shapes_agree_bit_for_bit(n, p, m, dev_block, slices, monkeypatch):
    # the register-staged shape (0), the shapes that load straight into LDS
    # (1, and 2 with wider waves) and the paired-digit shapes (3 staged
    # through registers, 4 to 6 loaded straight into three or two LDS
    # buffers, 6 with 128-byte stages: two digits per accumulator against
    # centred dosages, plus row sums) form
    # the same exact integers per digit pair, so their results are equal
    # bit for bit; strided device dosages with garbage past n give the same
    # bits as compact ones
    import torch
    seed = 61 + n
    prob = synth.make_problem(n, p, seed, k=max(50, n // 2))
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    dev = torch.device("cuda:0")
    ldx = (n + 15) // 16 * 16 + 48
    big = torch.full((m, ldx), 113, dtype=torch.int8, device=dev)
    big[:, :n] = torch.from_numpy(XR).to(dev)
    ref = None
    for cfg in TILE_SHAPES["int8"]:
        monkeypatch.setenv("GWAS_TRMM_CFG", str(cfg))
        _say(f"int8 slices={slices} shape {cfg} n={n} p={p} m={m} dev_block={dev_block}")
        kw = dict(precision="int8", x_dtype="i8", slices=slices, dev_block=dev_block)
        b, var, info = run(prob, XR, **kw)
        bs, vs, is_ = run(prob, big[:, :n], **kw)
        assert np.array_equal(b, bs.cpu().numpy()) and np.array_equal(var, vs.cpu().numpy())
        if ref is None:
            bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
            assert np.array_equal(info, io)
            err = normwise(b[io == 0], bo[io == 0])
            _say(f"  normwise {err:.3e} against the oracle")
            assert err < ({4: 1e-7, 5: 1e-9}.get(slices, TOL_FP64))
            ref = (b, var, info)
        else:
            assert np.array_equal(b, ref[0]) and np.array_equal(var, ref[1]) and np.array_equal(info, ref[2])


@pytest.mark.parametrize("n,m,dev_block", [(1030, 700, 256), (9000, 300, 128)])
def test_int8_dosages_outside_0_1_2(n, m, dev_block, monkeypatch):
    # The unpaired shape (0) sums any int8 dosage exactly and matches the
    # oracle; the paired shapes (3-5, centred dosages) cannot represent a
    # dosage outside {0, 1, 2}, so such SNPs come back NaN and every other
    # SNP keeps the unpaired shape's bits
    p, seed = 4, 401
    prob = synth.make_problem(n, p, seed, k=max(50, n // 2))
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    rng = np.random.default_rng(seed)
    bad = np.zeros(m, dtype=bool)
    bad[rng.choice(m, size=m // 10, replace=False)] = True
    vals = np.array([3, -1, 127, -128, 5], dtype=np.int8)
    for i in np.flatnonzero(bad):
        XR[i, rng.integers(0, n)] = vals[rng.integers(0, len(vals))]
    bad[-1] = True
    XR[-1, n - 1] = 3                              # in the last stage and the last column
    kw = dict(precision="int8", x_dtype="i8", dev_block=dev_block)
    monkeypatch.setenv("GWAS_TRMM_CFG", "0")
    _say(f"int8 dosages outside 0..2, shape 0, n={n} m={m}")
    b0, v0, i0 = run(prob, XR, **kw)
    bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    assert np.array_equal(i0, io) and normwise(b0[io == 0], bo[io == 0]) < TOL_FP64
    for cfg in (3, 4, 5, 6):
        monkeypatch.setenv("GWAS_TRMM_CFG", str(cfg))
        _say(f"  paired shape {cfg}")
        b, var, info = run(prob, XR, **kw)
        assert np.all(np.isnan(b[bad])) and np.all(np.isnan(var[bad]))
        assert np.array_equal(b[~bad], b0[~bad]) and np.array_equal(var[~bad], v0[~bad])
        assert np.array_equal(info[~bad], i0[~bad])


def test_int8_slices_needs_int8_dosages():
    prob = synth.make_problem(100, 3, 1)
    with pytest.raises(binding.GwasError) as ei:
        binding.GwasContext(prob["M"], prob["XL"], prob["Y"], precision="int8", x_dtype="f64")
    assert ei.value.code == 1


def _cohort_contexts(precision, dev_block, t=3, p=4, ns=(700, 1300, 2100)):
    probs = [synth.make_problem(n, p, 50 + i, t=t, k=400) for i, n in enumerate(ns)]
    xd = "i8"
    ctxs = [binding.GwasContext(pr["M"], pr["XL"], pr["Y"], precision=precision, x_dtype=xd,
                                dev_block=dev_block) for pr in probs]
    return probs, ctxs


@pytest.mark.parametrize("precision", ["fp64", "fp32", "int8"])
def test_group_matches_single_contexts(precision):
    m = 1500
    _say(f"group of 3 cohorts ({precision}), m={m}, ragged sub-blocks")
    probs, ctxs = _cohort_contexts(precision, dev_block=512)
    XRs = [synth.snp_block(pr["n"], 9, 0, m, dtype=np.int8, cohort=i) for i, pr in enumerate(probs)]
    try:
        grouped = binding.stream_group(ctxs, XRs)
        for c, X, (b, v, info) in zip(ctxs, XRs, grouped):
            b1, v1, i1 = c.stream_block(X)
            assert np.array_equal(b, b1) and np.array_equal(v, v1) and np.array_equal(info, i1)
        if precision == "fp64":
            for pr, X, (b, _, _) in zip(probs, XRs, grouped):
                bo, _, _ = GLSOracle(pr["M"], pr["XL"], pr["Y"]).solve(X)
                assert normwise(b, bo) < TOL_FP64
    finally:
        for c in ctxs:
            c.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "int8", "bf16x3"])
def test_group_graph_replays_match_eager(precision):
    # the reduced modes' graphs also hold the cross products and, for the
    # cohort of n = 2,100 (two K splits), the reduction of their partial sums;
    # the dosages of each call are new device tensors, which the replay reads
    # in place through its argument array
    import torch
    dev = torch.device("cuda:0")
    blk, m = 256, 1024
    _say(f"group graph {precision}: 3 cohorts, {m // blk} full sub-blocks per call, two calls")
    probs, ctxs = _cohort_contexts(precision, dev_block=blk)
    try:
        for call in range(2):
            XRs = [synth.snp_block_device(pr["n"], 10 + call, 0, m, dev, cohort=i)
                   for i, pr in enumerate(probs)]
            eager = binding.stream_group(ctxs, XRs)
            torch.cuda.synchronize()
            replay = binding.stream_group(ctxs, XRs, graph=True)
            torch.cuda.synchronize()
            for (be, ve, ie), (bg, vg, ig) in zip(eager, replay):
                assert torch.equal(be, bg) and torch.equal(ve, vg) and torch.equal(ie, ig)
            # eager work of the program between replays
            _ = [c.stream_block(X[:100]) for c, X in zip(ctxs, XRs)]
    finally:
        for c in ctxs:
            c.close()


def test_group_graph_after_a_member_is_replaced():
    # A captured group graph must not be replayed for a new context, even one
    # created at the freed member's address: the new member's buffers differ.
    import torch
    dev = torch.device("cuda:0")
    blk, m = 256, 512
    probs, ctxs = _cohort_contexts("fp64", dev_block=blk)
    try:
        XRs = [synth.snp_block_device(pr["n"], 21, 0, m, dev, cohort=i) for i, pr in enumerate(probs)]
        binding.stream_group(ctxs, XRs, graph=True)
        torch.cuda.synchronize()
        old = ctxs[1]._h.value
        ctxs[1].close()
        pr = probs[1]
        ctxs[1] = binding.GwasContext(pr["M"], pr["XL"], pr["Y"] * 2.0, x_dtype="i8", dev_block=blk)
        _say(f"replaced member at {old:#x} by one at {ctxs[1]._h.value:#x}")
        eager = binding.stream_group(ctxs, XRs)
        torch.cuda.synchronize()
        replay = binding.stream_group(ctxs, XRs, graph=True)
        torch.cuda.synchronize()
        for (be, ve, ie), (bg, vg, ig) in zip(eager, replay):
            assert torch.equal(be, bg) and torch.equal(ve, vg) and torch.equal(ie, ig)
        single = ctxs[1].stream_block(XRs[1])[0]
        assert torch.equal(single, replay[1][0])
    finally:
        for c in ctxs:
            c.close()


def test_group_rebuilt_after_autotune_changes_tile_height(tmp_path, monkeypatch):
    # Grouped schedules and graphs belong to the members' tile shape: after
    # gwas_autotune moves every member from 256-row tiles (shape 4) to 128-row
    # tiles (shape 2), eager and graph grouped calls must equal fresh
    # contexts built in shape 2, bit for bit.
    import torch
    dev = torch.device("cuda:0")
    blk, m = 512, 1024
    monkeypatch.setenv("GWAS_TRMM_CFG", "4")
    probs, ctxs = _cohort_contexts("fp64", dev_block=blk)
    monkeypatch.setenv("GWAS_TRMM_CFG", "2")
    _, fresh = _cohort_contexts("fp64", dev_block=blk)
    monkeypatch.delenv("GWAS_TRMM_CFG")
    cache = tmp_path / "tune.txt"
    # cache lines that make each member's autotune choose shape 2, row group 1
    cache.write_text("".join(f"gfx950 n_pad={c.query()['n_pad']} precision=0 x_dtype=1 cols={blk} cfg=2 rgroup=1\n"
                             for c in ctxs))
    monkeypatch.setenv("GWAS_TUNE_CACHE", str(cache))
    try:
        XRs = [synth.snp_block_device(pr["n"], 31, 0, m, dev, cohort=i) for i, pr in enumerate(probs)]
        binding.stream_group(ctxs, XRs)
        binding.stream_group(ctxs, XRs, graph=True)
        torch.cuda.synchronize()
        for c, X in zip(ctxs, XRs):
            assert c.autotune(X, blk) == (2, 1)
        ref = binding.stream_group(fresh, XRs)
        after = binding.stream_group(ctxs, XRs)
        torch.cuda.synchronize()
        replay = binding.stream_group(ctxs, XRs, graph=True)
        torch.cuda.synchronize()
        _say("group after autotune 4 -> 2: eager and graph calls against fresh shape-2 contexts")
        for r, a, g in zip(ref, after, replay):
            for x, y, z in zip(r, a, g):
                assert torch.equal(x, y) and torch.equal(x, z)
    finally:
        for c in ctxs + fresh:
            c.close()


def test_autotune_and_cache(tmp_path, monkeypatch):
    n, p, m, seed = 1500, 4, 2048, 61
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    bo, _, _ = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("GWAS_TUNE_CACHE", str(cache))
    for precision, tol in [("fp64", TOL_FP64), ("fp32", TOL_FP32), ("int8", TOL_FP64)]:
        with binding.GwasContext(prob["M"], prob["XL"], prob["Y"], precision=precision, x_dtype="i8",
                                 dev_block=1024) as ctx:
            best = ctx.autotune(XR, 1024)
            sub = ctx.query()["dev_block"]
            _say(f"autotune {precision}: tile shape {best[0]}, row group {best[1]}, sub-block width {sub}")
            assert best[0] in TILE_SHAPES[precision] and best[1] in (1, 2, 4, 8) and sub in (256, 512, 1024)
            b, _, _ = ctx.stream_block(XR)
            assert normwise(b, bo) < tol
        with binding.GwasContext(prob["M"], prob["XL"], prob["Y"], precision=precision, x_dtype="i8",
                                 dev_block=1024) as ctx:
            assert ctx.autotune(XR, 1024) == best          # read back from the cache
            assert ctx.query()["dev_block"] == sub
            b2, _, _ = ctx.stream_block(XR)
            assert torch_equal(b, b2)                      # same shape and schedule: same bits
    lines = cache.read_text().splitlines()
    assert len(lines) == 3 and all("cfg=" in ln and "rgroup=" in ln and "sub=" in ln for ln in lines)


def test_many_traits():
    n, p, t, m, seed = 1500, 4, 64, 600, 71
    _say(f"traits n={n} p={p} t={t} m={m}")
    prob = synth.make_problem(n, p, seed, t=t)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    for precision, tol in [("fp64", TOL_FP64), ("int8", TOL_FP64), ("fp32", TOL_FP32)]:
        b, var, info = run(prob, XR, precision=precision, x_dtype="i8")
        err = normwise(b, bo)
        _say(f"  {precision}: err {err:.3e}")
        assert b.shape == (m, t, p) and err < tol


@pytest.mark.parametrize("precision,x_dtype,tol", [("fp32", "f64", TOL_FP32), ("fp32", "i8", TOL_FP32),
                                                   ("int8", "i8", TOL_FP64)])
def test_cross_products_k_splits_and_wide_w(precision, x_dtype, tol):
    # The reduced-precision modes form x_i^T [W_L | w_y] on their own: odd n
    # past two K splits of 2,048 rows (the last one ragged), p-1+t = 82
    # columns of W (past the 80 one workgroup takes) and a ragged SNP tile.
    n, p, t, m, seed = 4099, 3, 80, 300, 83
    _say(f"cross products {precision} x={x_dtype} n={n} p={p} t={t} m={m}")
    prob = synth.make_problem(n, p, seed, t=t)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8 if x_dtype == "i8" else np.float64)
    bo, vo, io = GLSOracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    b, var, info = run(prob, XR, precision=precision, x_dtype=x_dtype, dev_block=512)
    assert np.array_equal(info, io)
    err = normwise(b, bo)
    _say(f"  err {err:.3e}")
    assert b.shape == (m, t, p) and err < tol


@pytest.mark.parametrize("precision", ["fp32", "int8", "fp64"])
def test_wide_stride_device_dosages_are_staged(precision):
    # A device array whose columns are 9 MB apart: 256 such columns span
    # more than 2^31 bytes, past the 32-bit offsets of the products' buffer
    # loads, so the library stages the block and gives the compact input's
    # result bit for bit.
    import torch
    n, p, m, seed, ldx = 300, 4, 3, 47, 9_000_000
    _say(f"wide stride {precision} n={n} m={m} ldx={ldx}")
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    dev = torch.device("cuda:0")
    big = torch.zeros((m, ldx), dtype=torch.int8, device=dev)
    big[:, :n] = torch.from_numpy(XR).to(dev)
    wide = big[:, :n]
    assert wide.stride(0) == ldx
    kw = dict(precision=precision, x_dtype="i8")
    b0, v0, i0 = run(prob, torch.from_numpy(XR).to(dev).contiguous(), **kw)
    b1, v1, i1 = run(prob, wide, **kw)
    torch.cuda.synchronize()
    assert torch_equal(i0.cpu(), i1.cpu())
    assert torch_equal(b0.cpu(), b1.cpu()) and torch_equal(v0.cpu(), v1.cpu())


@pytest.mark.parametrize("precision", ["fp32", "bf16", "int8"])
def test_reduced_precision_partition_independence(precision):
    # A SNP lands at a different row of the matrix-core tiles (product and
    # cross products) depending on its offset in the block; its bits must
    # not change.  n spans two K splits of the cross products.
    n, p, m, seed = 2500, 4, 1200, 37
    _say(f"partition {precision} n={n} p={p} m={m}")
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    kw = dict(precision=precision, x_dtype="i8")
    b1, v1, i1 = run(prob, XR, dev_block=256, **kw)
    b2, v2, i2 = run(prob, XR, dev_block=1024, **kw)
    assert np.array_equal(i1, i2)
    assert np.array_equal(b1, b2) and np.array_equal(v1, v2)
    with binding.GwasContext(prob["M"], prob["XL"], prob["Y"], dev_block=512, **kw) as ctx:
        parts = [ctx.stream_block(XR[a:b_])[0] for a, b_ in [(0, 1), (1, 333), (333, m)]]
    assert np.array_equal(np.concatenate(parts), b1)


@pytest.mark.parametrize("precision,x_dtype,tol", [("fp64", "f64", TOL_FP64), ("fp64", "i8", TOL_FP64),
                                                   ("fp32", "i8", TOL_FP32), ("int8", "i8", TOL_FP64)])
def test_p2_intercept_only(precision, x_dtype, tol):
    # p = 2: X_L is the intercept alone, the smallest instance of every
    # per-SNP kernel (one covariate, one cross term, a 2 x 2 solve).
    n, p, m, seed = 513, 2, 300, 89
    _say(f"p=2 {precision} x={x_dtype} n={n} m={m}")
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8 if x_dtype == "i8" else np.float64)
    b, var, info = run(prob, XR, precision=precision, x_dtype=x_dtype, dev_block=256)
    orc = GLSOracle(prob["M"], prob["XL"], prob["Y"])
    bo, vo, io = orc.solve(XR)
    assert np.array_equal(info, io) and b.shape == (m, 1, p)
    if precision == "fp32":
        # at n this small the float32 rounding of L^-1, magnified by the
        # cancellation in S_BR - S_BL S_TL^-1 S_BL^T, reaches 1e-8 (2e-8 at
        # n = 130): each SNP is held to twice its first-order rounding bound,
        # as in the ragged small-n test, and the block to 5e-8
        ok = io == 0
        bound = rounding_bound(prob, XR[ok], bo[ok], 2.0 ** -24, 2.0 ** -24)
        num = np.linalg.norm((b[ok] - bo[ok]).reshape(int(ok.sum()), -1), axis=1)
        rel = num / np.linalg.norm(bo[ok].reshape(int(ok.sum()), -1), axis=1)
        srel, vrel, se = snp_errors(b, bo, var, vo, ok)
        worst, kmax = reduced_floor(orc, XR, b, bo, var, vo, ok, U32)
        _say(f"  err {rel.max():.3e}, worst err / bound {np.max(rel / (bound + 1e-300)):.3f}; "
             f"SNP coefficient rel {srel:.3e} ({se:.3e} SE), var rel {vrel:.3e}, "
             f"against 16 u kappa {worst:.3f} (kappa <= {kmax:.1f})")
        assert np.all(rel <= 2.0 * bound + 1e-13) and worst <= 1.0
        return
    err = normwise(b, bo)
    verr = float(np.max(np.abs(var - vo) / np.abs(vo)))
    _say(f"  err {err:.3e} var err {verr:.3e}")
    assert err < tol and verr < 1e-10


def _random_configs(count=24, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        precision = ["fp64", "fp32", "int8"][k % 3]
        n = int(rng.integers(2, 3001))
        p = int(rng.integers(2, min(20, n) + 1))
        t = int(rng.choice([1, 1, 2, 5]))
        m = int(rng.integers(1, 1201))
        dev_block = int(rng.choice([128, 256, 384, 512, 1024]))
        x_dtype = "i8" if precision == "int8" else str(rng.choice(["f64", "i8"]))
        on_device = bool(rng.integers(0, 2))
        out.append((precision, n, p, t, m, dev_block, x_dtype, on_device))
    return out


@pytest.mark.parametrize("precision,n,p,t,m,dev_block,x_dtype,on_device", _random_configs())
def test_random_shapes_vs_oracle(precision, n, p, t, m, dev_block, x_dtype, on_device):
    # Seeded random shapes across precision, n, p, traits, block width,
    # dosage type and host or device inputs and outputs.
    import torch
    seed = 1000 + n + 7 * p + m
    _say(f"random {precision} n={n} p={p} t={t} m={m} dev_block={dev_block} x={x_dtype} device={on_device}")
    prob = synth.make_problem(n, p, seed, t=t, k=max(50, n // 2))
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8 if x_dtype == "i8" else np.float64)
    kw = dict(precision=precision, x_dtype=x_dtype, dev_block=dev_block)
    if on_device:
        dev = torch.device("cuda:0")
        with binding.GwasContext(torch.from_numpy(prob["M"]).to(dev), torch.from_numpy(prob["XL"]).to(dev),
                                 torch.from_numpy(prob["Y"]).to(dev), **kw) as ctx:
            b, var, info = ctx.stream_block(torch.from_numpy(XR).to(dev))
            torch.cuda.synchronize()
            b, var, info = b.cpu().numpy(), var.cpu().numpy(), info.cpu().numpy()
    else:
        b, var, info = run(prob, XR, **kw)
    orc = GLSOracle(prob["M"], prob["XL"], prob["Y"])
    bo, vo, io = orc.solve(XR)
    assert np.array_equal(info, io)
    ok = io == 0
    assert b.shape == (m, t, p)
    if not ok.any():
        return
    num = np.linalg.norm((b[ok] - bo[ok]).reshape(int(ok.sum()), -1), axis=1)
    rel = num / np.linalg.norm(bo[ok].reshape(int(ok.sum()), -1), axis=1)
    if precision == "fp32":
        # each trait against its own first-order rounding bound (small n)
        worst = 0.0
        for j in range(t):
            bj, boj = b[ok][:, j, :], bo[ok][:, j, :]
            relj = np.linalg.norm(bj - boj, axis=1) / np.linalg.norm(boj, axis=1)
            bound = rounding_bound(prob, XR[ok], bo[ok][:, j:j + 1, :], 2.0 ** -24, 2.0 ** -24)
            worst = max(worst, float(np.max(relj / (bound + 1e-300))))
            assert np.all(relj <= 2.0 * bound + 1e-13)
        srel, vrel, se = snp_errors(b, bo, var, vo, ok)
        fl, kmax = reduced_floor(orc, XR, b, bo, var, vo, ok, U32)
        _say(f"  err {rel.max():.3e}, worst err / bound {worst:.3f}; SNP coefficient rel {srel:.3e} "
             f"({se:.3e} SE), var rel {vrel:.3e}, against 16 u kappa {fl:.3f} (kappa <= {kmax:.1f})")
        assert fl <= 1.0
    else:
        tol = TOL_FP64 if (precision == "fp64" or n >= 100) else 1e-8
        srel, vrel, se = snp_errors(b, bo, var, vo, ok)
        _say(f"  err {rel.max():.3e}; SNP coefficient {se:.3e} SE, var rel {vrel:.3e}")
        assert rel.max() < tol and se < tol


def _random_groups(count=8, seed=2025):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        precision = ["fp64", "fp32", "int8"][k % 3]
        nctx = int(rng.integers(2, 6))
        shapes = []
        for _ in range(nctx):
            n = int(rng.integers(50, 3001))
            shapes.append((n, int(rng.integers(2, 9)), int(rng.choice([1, 2, 3]))))
        dev_block = int(rng.choice([128, 256, 512]))
        graph = k % 2 == 1
        # graph replay covers full-width sub-blocks: give those groups some
        m = (dev_block * int(rng.integers(1, 4)) + int(rng.integers(0, dev_block))) if graph \
            else int(rng.integers(1, 1500))
        on_device = bool(rng.integers(0, 2))
        out.append((precision, tuple(shapes), m, dev_block, graph, on_device))
    return out


@pytest.mark.parametrize("precision,shapes,m,dev_block,graph,on_device", _random_groups())
def test_random_groups_match_single_contexts(precision, shapes, m, dev_block, graph, on_device):
    # Seeded random groups: contexts of their own n, p and traits, one width,
    # eager or graph replay, host or device data; each member's result equals
    # its own single-context call bit for bit.
    import torch
    _say(f"random group {precision} shapes={shapes} m={m} dev_block={dev_block} graph={graph} device={on_device}")
    dev = torch.device("cuda:0")
    probs = [synth.make_problem(n, p, 300 + i, t=t, k=max(50, n // 2)) for i, (n, p, t) in enumerate(shapes)]
    XRs = [synth.snp_block(pr["n"], 77, 0, m, dtype=np.int8, cohort=i) for i, pr in enumerate(probs)]
    if on_device:
        XRs = [torch.from_numpy(X).to(dev) for X in XRs]
    ctxs = [binding.GwasContext(pr["M"], pr["XL"], pr["Y"], precision=precision, x_dtype="i8", dev_block=dev_block)
            for pr in probs]
    try:
        single = [c.stream_block(X) for c, X in zip(ctxs, XRs)]
        for rep in range(2 if graph else 1):
            grouped = binding.stream_group(ctxs, XRs, graph=graph)
            if on_device:
                torch.cuda.synchronize()
            for (bs, vs, is_), (bg, vg, ig) in zip(single, grouped):
                eq = (torch.equal if on_device else np.array_equal)
                assert eq(bs, bg) and eq(vs, vg) and eq(is_, ig)
    finally:
        for c in ctxs:
            c.close()


def _random_queues(count=6, seed=2027):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        precision = ["fp64", "fp32", "int8"][k % 3]
        n = int(rng.integers(50, 3001))
        p = int(rng.integers(2, 9))
        m = int(rng.integers(200, 2500))
        cuts = tuple(sorted(int(x) for x in rng.choice(np.arange(1, m), size=int(rng.integers(1, 7)), replace=False)))
        x_dtype = "i8" if precision == "int8" else str(rng.choice(["f64", "i8"]))
        out.append((precision, n, p, m, cuts, int(rng.choice([128, 256, 512])), x_dtype, bool(rng.integers(0, 2))))
    return out


@pytest.mark.parametrize("precision,n,p,m,cuts,dev_block,x_dtype,on_device", _random_queues())
def test_random_queued_blocks_match_one_call(precision, n, p, m, cuts, dev_block, x_dtype, on_device):
    # A block cut at random points and handed over as queued blocks (every
    # third one synchronously) gives the bits of one synchronous call.
    import torch
    _say(f"random queue {precision} n={n} p={p} m={m} cuts={cuts} dev_block={dev_block} x={x_dtype} "
         f"device={on_device}")
    prob = synth.make_problem(n, p, 600 + n)
    XR = synth.snp_block(n, 600 + n, 0, m, dtype=np.int8 if x_dtype == "i8" else np.float64)
    dev = torch.device("cuda:0")
    X = torch.from_numpy(XR).to(dev) if on_device else torch.from_numpy(XR).pin_memory()
    kw = dict(precision=precision, x_dtype=x_dtype, dev_block=dev_block)
    bounds = [0, *cuts, m]
    with binding.GwasContext(prob["M"], prob["XL"], prob["Y"], **kw) as ctx:
        ref = ctx.stream_block(X)
        outs = []
        for j, (a, e) in enumerate(zip(bounds[:-1], bounds[1:])):
            o = ctx._outputs(e - a, on_device, dev)
            if not on_device:
                o = tuple(torch.from_numpy(t).pin_memory() for t in o)
            if j % 3 == 2:
                ctx.stream_block(X[a:e], out=o)
            else:
                ctx.stream_block_async(X[a:e], o)
            outs.append(o)
        ctx.wait()
    if on_device:
        torch.cuda.synchronize()
    for k in range(3):
        got = torch.cat([o[k] for o in outs]).cpu()
        want = ref[k].cpu() if on_device else torch.from_numpy(np.asarray(ref[k]))
        assert torch.equal(got, want)
