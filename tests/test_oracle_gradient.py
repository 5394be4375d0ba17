"""Pins for the reverse-mode oracle: central finite differences of the
(pinned) forward oracle, and the closed form of the Wald-loss gradient
d/dy = 2 P X_R b_SNP with P = M^-1 - M^-1 X_L (X_L^T M^-1 X_L)^-1 X_L^T M^-1.
CPU only."""

import numpy as np

from oracle import gradient as og
from paper_1304_2272_amd import synth


def _case(n=120, p=4, m=30, seed=3, h2=0.45, sigma2=1.3):
    Z = synth.background_genotypes(n, seed, k=60)
    Phi = Z @ Z.T / Z.shape[1]
    rng = np.random.default_rng(seed)
    XL = np.column_stack([np.ones(n), rng.standard_normal((n, p - 2))])
    y = rng.standard_normal(n)
    XR = synth.snp_block(n, seed, 0, m)
    return Phi, sigma2, h2, XL, y, XR


def test_wald_gradient_matches_central_differences():
    Phi, s2, h2, XL, y, XR = _case()
    loss, gy, gh2 = og.wald_gradient(Phi, s2, h2, XL, y, XR)
    d = 1e-6
    fd_h2 = (og.wald_loss(og.model_covariance(Phi, s2, h2 + d), XL, y, XR) -
             og.wald_loss(og.model_covariance(Phi, s2, h2 - d), XL, y, XR)) / (2 * d)
    assert abs(gh2 - fd_h2) < 1e-6 * max(1.0, abs(fd_h2))
    M = og.model_covariance(Phi, s2, h2)
    rng = np.random.default_rng(7)
    for _ in range(3):
        v = rng.standard_normal(y.shape[0])
        v /= np.linalg.norm(v)
        fd = (og.wald_loss(M, XL, y + d * v, XR) - og.wald_loss(M, XL, y - d * v, XR)) / (2 * d)
        assert abs(gy @ v - fd) < 1e-5 * max(1.0, abs(fd))


def test_wald_gradient_closed_form_in_y():
    Phi, s2, h2, XL, y, XR = _case(seed=5)
    loss, gy, _ = og.wald_gradient(Phi, s2, h2, XL, y, XR)
    M = og.model_covariance(Phi, s2, h2)
    Minv = np.linalg.inv(M)
    P = Minv - Minv @ XL @ np.linalg.inv(XL.T @ Minv @ XL) @ XL.T @ Minv
    bs = (XR @ P @ y) / np.einsum("in,nk,ik->i", XR, P, XR)
    assert np.allclose(gy, 2 * P @ XR.T @ bs, rtol=1e-10, atol=1e-12)
    assert abs(loss - np.sum(bs * (XR @ P @ y))) < 1e-10 * loss


def test_generic_cotangents_match_differences():
    # an arbitrary loss of b and var: l = sum_i w_i . b_i + c_i var_i
    Phi, s2, h2, XL, y, XR = _case(n=90, m=12, seed=11)
    rng = np.random.default_rng(2)
    W = rng.standard_normal((XR.shape[0], XL.shape[1] + 1))
    C = rng.standard_normal(XR.shape[0])
    from oracle import GLSOracle

    def loss(M, yy):
        b, var, _ = GLSOracle(M, XL, yy).solve(XR)
        return float(np.sum(W * b[:, 0, :]) + np.sum(C * var))

    M = og.model_covariance(Phi, s2, h2)
    gy, Mbar = og.reverse(M, XL, y, XR, W, C)
    d = 1e-6
    fd = (loss(og.model_covariance(Phi, s2, h2 + d), y) - loss(og.model_covariance(Phi, s2, h2 - d), y)) / (2 * d)
    assert abs(np.sum(Mbar * s2 * (Phi - np.eye(Phi.shape[0]))) - fd) < 1e-6 * max(1.0, abs(fd))
    v = rng.standard_normal(y.shape[0])
    fdy = (loss(M, y + d * v) - loss(M, y - d * v)) / (2 * d)
    assert abs(gy @ v - fdy) < 1e-6 * max(1.0, abs(fdy))


def test_contracted_gradient_equals_dense():
    """The batched form used at n = 10^4 reproduces the dense-dl/dM oracle."""
    from oracle import gradient as og
    n, p, m, seed = 240, 4, 60, 9
    Z = synth.background_genotypes(n, seed, k=300)
    Phi = Z @ Z.T / Z.shape[1]
    prob = synth.make_problem(n, p, seed, k=300)
    XR = synth.snp_block(n, seed, 0, m)
    l0, gy0, gh0 = og.wald_gradient(Phi, 1.3, 0.41, prob["XL"], prob["Y"][:, 0], XR)
    l1, gy1, gh1 = og.wald_gradient_contracted(Phi, 1.3, 0.41, prob["XL"], prob["Y"][:, 0], XR)
    assert abs(l1 - l0) <= 1e-11 * abs(l0)
    assert np.max(np.abs(gy1 - gy0)) <= 1e-10 * np.max(np.abs(gy0))
    assert abs(gh1 - gh0) <= 1e-10 * abs(gh0)


def test_scale_of_M_closed_form():
    """b does not change when M is scaled and var scales with it, so the
    Wald loss is l(c M) = l(M) / c and <dl/dM, M> = d l(c M)/dc at c = 1 = -l."""
    Phi, s2, h2, XL, y, XR = _case(seed=11)
    M = og.model_covariance(Phi, s2, h2)
    b, var, _ = og.GLSOracle(M, XL, y).solve(XR)
    gb, gv = og.wald_loss_cotangents(b, var)
    _, Mbar = og.reverse(M, XL, y, XR, gb, gv)
    loss = og.wald_loss(M, XL, y, XR)
    assert abs(np.sum(Mbar * M) + loss) < 1e-9 * loss
