"""GPU reverse pass against the reverse-mode oracle and finite differences."""

import numpy as np
import pytest

from oracle import gradient as og
from paper_1304_2272_amd import binding, synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _case(n, p, m, seed, h2=0.5, sigma2=1.0, dtype=np.float64):
    Z = synth.background_genotypes(n, seed, k=min(2000, 2 * n))
    Phi = Z @ Z.T / Z.shape[1]
    prob = synth.make_problem(n, p, seed, k=min(2000, 2 * n))
    XR = synth.snp_block(n, seed, 0, m, dtype=dtype)
    return Phi, sigma2, h2, prob["XL"], prob["Y"][:, 0], XR


@pytest.fixture(scope="module", autouse=True)
def _lib():
    binding.load()


def _contraction_errors(tr, ip, Mbar, M):
    """Errors of tr Mbar and <Mbar, M> against the oracle's dense adjoint,
    each relative to the sum of the magnitudes of its own terms (the scale
    of the rounding in either sum)."""
    etr = abs(tr - np.trace(Mbar)) / np.abs(np.diag(Mbar)).sum()
    eip = abs(ip - np.sum(Mbar * M)) / np.abs(Mbar * M).sum()
    return etr, eip


@pytest.mark.parametrize("x_dtype,p", [("f64", 4), ("i8", 4), ("f64", 2), ("i8", 7)])
def test_reverse_generic_cotangents_vs_oracle(x_dtype, p):
    # p = 2 is the smallest instance of the per-SNP reverse kernel
    n, m = 300, 700
    _say(f"reverse pass, random cotangents, n={n} p={p} m={m} x={x_dtype}")
    Phi, s2, h2, XL, y, XR = _case(n, p, m, 21, dtype=np.int8 if x_dtype == "i8" else np.float64)
    M = og.model_covariance(Phi, s2, h2)
    rng = np.random.default_rng(4)
    gb = rng.standard_normal((m, p))
    gv = rng.standard_normal(m)
    with binding.GwasContext(M, XL, y, x_dtype=x_dtype, dev_block=256) as ctx:
        b, var, info = ctx.stream_block(XR)
        ctx.backward_begin()
        ctx.backward_block(XR, b[:, 0, :], var, info, gb, gv)
        gy, tr, ip = ctx.backward_end()
    gy_o, Mbar = og.reverse(M, XL, y, XR, gb, gv)
    rel = np.max(np.abs(gy - gy_o)) / np.max(np.abs(gy_o))
    etr, eip = _contraction_errors(tr, ip, Mbar, M)
    _say(f"  dl/dy rel err {rel:.2e}; tr {tr:.6e} vs {np.trace(Mbar):.6e}; <Mbar,M> {ip:.6e} vs {np.sum(Mbar * M):.6e}"
         f"; errors {etr:.2e} of sum |Mbar_jj|, {eip:.2e} of sum |Mbar_ij M_ij|")
    assert rel < 1e-12
    assert etr < 1e-12 and eip < 1e-13


def test_autograd_wald_loss_vs_oracle():
    import torch
    from paper_1304_2272_amd.autograd import GwasGLS
    n, p, m = 1200, 4, 1500
    _say(f"autograd Wald loss n={n} p={p} m={m}")
    Phi, s2, h2, XL, y, XR = _case(n, p, m, 31, h2=0.37, sigma2=1.4)
    dev = torch.device("cuda:0")
    yt = torch.tensor(y, device=dev, requires_grad=True)
    h2t = torch.tensor(h2, dtype=torch.float64, device=dev, requires_grad=True)
    s2t = torch.tensor(s2, dtype=torch.float64, device=dev, requires_grad=True)
    b, var = GwasGLS.apply(yt, h2t, torch.tensor(Phi, device=dev), torch.tensor(XL, device=dev),
                           torch.tensor(XR, device=dev), s2t, {"dev_block": 512})
    loss = (b[:, -1] ** 2 / var).sum()
    loss.backward()
    lo, gyo, gho = og.wald_gradient(Phi, s2, h2, XL, y, XR)
    gy = yt.grad.cpu().numpy()
    _say(f"  loss {loss.item():.10e} vs {lo:.10e}; dh2 {h2t.grad.item():.10e} vs {gho:.10e}; "
         f"dsigma2 {s2t.grad.item():.10e} vs -loss/sigma2 {-lo / s2:.10e}")
    assert abs(loss.item() - lo) < 1e-10 * lo
    assert np.max(np.abs(gy - gyo)) < 1e-8 * np.max(np.abs(gyo))
    assert abs(h2t.grad.item() - gho) < 1e-8 * abs(gho)
    # b does not depend on sigma2 and var scales with it: dl/dsigma2 = -l / sigma2
    assert abs(s2t.grad.item() + lo / s2) < 1e-9 * abs(lo / s2)


@pytest.mark.parametrize("h2", [0.3, 0.02, 1e-3])
def test_dh2_at_small_heritability(h2):
    # dl/dh^2 = (<Mbar, M> - sigma^2 tr Mbar) / h^2: as h^2 -> 0 the two
    # contractions approach each other and the difference keeps the error of
    # each, so the relative error of dl/dh^2 grows like
    # A = (|<Mbar, M>| + sigma^2 |tr Mbar|) / (h^2 |dl/dh^2|).  The oracle
    # contracts Mbar with sigma^2 (Phi - I) directly; the library's value
    # must be within 1e-13 A of it, i.e. lose no more than that cancellation
    # (measured 1-2e-14 A at h^2 = 0.3, 0.02 and 0.001).
    n, p, m, s2 = 800, 4, 600, 1.3
    _say(f"dl/dh2 at h2={h2}, n={n} p={p} m={m}")
    Phi, _, _, XL, y, XR = _case(n, p, m, 41, h2=h2, sigma2=s2)
    M = og.model_covariance(Phi, s2, h2)
    lo, _, gho = og.wald_gradient(Phi, s2, h2, XL, y, XR)
    with binding.GwasContext(M, XL, y, dev_block=256) as ctx:
        b, var, info = ctx.stream_block(XR)
        gb, gv = og.wald_loss_cotangents(b, var)
        ctx.backward_begin()
        ctx.backward_block(XR, b[:, 0, :], var, info, gb, gv)
        _, tr, ip = ctx.backward_end()
    dh2 = (ip - s2 * tr) / h2
    A = (abs(ip) + s2 * abs(tr)) / (h2 * abs(gho))
    err = abs(dh2 - gho) / abs(gho)
    _say(f"  dh2 {dh2:.12e} vs oracle {gho:.12e}: rel err {err:.2e}, cancellation factor A = {A:.2e}")
    assert err < 1e-13 * A


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_n10000_gradient_vs_differences():
    import torch
    from paper_1304_2272_amd.autograd import GwasGLS
    n, p, m, seed = 10_000, 4, 100_000, 1309
    _say(f"n={n} p={p} m={m}: gradient vs central differences of the GPU forward")
    dev = torch.device("cuda:0")
    Z = torch.tensor(synth.background_genotypes(n, seed), device=dev)
    Phi = Z @ Z.t().contiguous() / Z.shape[1]
    del Z
    prob = synth.make_problem(n, p, seed)
    XL = torch.tensor(prob["XL"], device=dev)
    y0 = torch.tensor(prob["Y"][:, 0], device=dev)
    XR = synth.snp_block_device(n, seed, 0, m, dev)
    opts = {"x_dtype": "i8"}

    def loss_at(yv, h2v):
        with torch.no_grad():
            b, var = GwasGLS.apply(yv, torch.tensor(h2v, dtype=torch.float64, device=dev), Phi, XL, XR, 1.0, opts)
            return float((b[:, -1] ** 2 / var).sum())

    yt = y0.clone().requires_grad_(True)
    h2t = torch.tensor(0.5, dtype=torch.float64, device=dev, requires_grad=True)
    b, var = GwasGLS.apply(yt, h2t, Phi, XL, XR, 1.0, opts)
    loss = (b[:, -1] ** 2 / var).sum()
    loss.backward()
    d = 1e-6
    fd_h2 = (loss_at(y0, 0.5 + d) - loss_at(y0, 0.5 - d)) / (2 * d)
    _say(f"  loss {loss.item():.6e}; dh2 {h2t.grad.item():.8e} vs FD {fd_h2:.8e}")
    assert abs(h2t.grad.item() - fd_h2) < 1e-6 * abs(fd_h2)
    g = torch.Generator(device="cpu").manual_seed(seed)
    for k in range(4):
        v = torch.randn(n, generator=g, dtype=torch.float64).to(dev)
        v /= v.norm()
        fd = (loss_at(y0 + d * v, 0.5) - loss_at(y0 - d * v, 0.5)) / (2 * d)
        an = float(yt.grad @ v)
        _say(f"  direction {k}: dy.v {an:.8e} vs FD {fd:.8e}")
        assert abs(an - fd) < 1e-4 * max(abs(fd), 1e-3 * float(yt.grad.norm()))


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_n10000_gradient_vs_oracle_on_2000_snps():
    """The differentiation workload's shape (n = 10,000, p = 4, float64
    dosages) on a fixed 2,000-SNP subset, loss restricted to that subset:
    loss, dl/dy and dl/dh^2 against the oracle gradient."""
    import torch
    from paper_1304_2272_amd.autograd import GwasGLS
    n, p, m, seed, h2, s2 = 10_000, 4, 2000, 1310, 0.5, 1.0
    _say(f"n={n} p={p} m={m}: GPU reverse pass vs oracle gradient")
    Z = synth.background_genotypes(n, seed)
    Phi = Z @ Z.T / Z.shape[1]
    del Z
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m)
    dev = torch.device("cuda:0")
    yt = torch.tensor(prob["Y"][:, 0], device=dev, requires_grad=True)
    h2t = torch.tensor(h2, dtype=torch.float64, device=dev, requires_grad=True)
    b, var = GwasGLS.apply(yt, h2t, torch.tensor(Phi, device=dev), torch.tensor(prob["XL"], device=dev),
                           torch.tensor(XR, device=dev), s2, {})
    loss = (b[:, -1] ** 2 / var).sum()
    loss.backward()
    lo, gyo, gho = og.wald_gradient_contracted(Phi, s2, h2, prob["XL"], prob["Y"][:, 0], XR)
    gy = yt.grad.cpu().numpy()
    rel_y = np.max(np.abs(gy - gyo)) / np.max(np.abs(gyo))
    _say(f"  loss {loss.item():.10e} vs {lo:.10e}; dh2 {h2t.grad.item():.10e} vs {gho:.10e}; dl/dy rel {rel_y:.2e}")
    assert abs(loss.item() - lo) < 1e-10 * lo
    assert rel_y < 1e-8
    assert abs(h2t.grad.item() - gho) < 1e-8 * abs(gho)


def _random_reverse(count=8, seed=2026):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.integers(20, 2501))
        p = int(rng.integers(2, min(10, n) + 1))
        m = int(rng.integers(1, 801))
        x_dtype = ["f64", "i8"][k % 2]
        dev_block = int(rng.choice([128, 256, 512]))
        out.append((n, p, m, x_dtype, dev_block))
    return out


@pytest.mark.parametrize("n,p,m,x_dtype,dev_block", _random_reverse())
def test_random_reverse_vs_oracle(n, p, m, x_dtype, dev_block):
    # Seeded random shapes through the reverse pass: dl/dy, tr Mbar and
    # <Mbar, M> against the oracle's dense adjoint for random cotangents.
    _say(f"random reverse n={n} p={p} m={m} x={x_dtype} dev_block={dev_block}")
    Phi, s2, h2, XL, y, XR = _case(n, p, m, 500 + n, dtype=np.int8 if x_dtype == "i8" else np.float64)
    M = og.model_covariance(Phi, s2, h2)
    rng = np.random.default_rng(n + m)
    gb = rng.standard_normal((m, p))
    gv = rng.standard_normal(m)
    with binding.GwasContext(M, XL, y, x_dtype=x_dtype, dev_block=dev_block) as ctx:
        b, var, info = ctx.stream_block(XR)
        ctx.backward_begin()
        ctx.backward_block(XR, b[:, 0, :], var, info, gb, gv)
        gy, tr, ip = ctx.backward_end()
    gy_o, Mbar = og.reverse(M, XL, y, XR, gb, gv)
    rel = np.max(np.abs(gy - gy_o)) / np.max(np.abs(gy_o))
    etr, eip = _contraction_errors(tr, ip, Mbar, M)
    _say(f"  dl/dy rel err {rel:.2e}; tr err {etr:.2e} of sum |Mbar_jj|, <Mbar,M> err {eip:.2e} of sum |Mbar_ij M_ij|")
    assert rel < 1e-12
    assert etr < 1e-12 and eip < 1e-13
