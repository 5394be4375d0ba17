"""CPU oracle for the reverse mode of the GLS solves of Eq. (1).

TEST INFRASTRUCTURE ONLY (see ``oracle/gls.py``).

For a scalar loss l(b, var) of the per-SNP solutions b_i = S_i^-1 r_i
(S_i = X_i^T M^-1 X_i, r_i = X_i^T M^-1 y) and of var_i = [S_i^-1]_pp, with
cotangents gb_i = dl/db_i and gv_i = dl/dvar_i, the derivatives follow from
d(M^-1) = -M^-1 dM M^-1 written out with dense matrices:

    dl/dy = sum_i M^-1 X_i S_i^-1 gb_i
    dl/dM = -sum_i sym(f_i e_i^T) + sum_i gv_i t_i t_i^T,
            f_i = M^-1 X_i S_i^-1 gb_i,  e_i = M^-1 (y - X_i b_i),
            t_i = M^-1 X_i S_i^-1 e_p

and, for M = sigma^2 (h^2 Phi + (1 - h^2) I), dl/dh^2 = <dl/dM, sigma^2 (Phi - I)>.
Everything is float64 with an explicit inverse of M (numpy), for small n.
"""

from __future__ import annotations

import numpy as np

from .gls import GLSOracle


def model_covariance(Phi, sigma2, h2):
    n = Phi.shape[0]
    return sigma2 * (h2 * Phi + (1.0 - h2) * np.eye(n))


def wald_loss_cotangents(b, var):
    """l = sum_i b_SNP,i^2 / var_i (one trait): (gb, gv)."""
    bs = b[:, 0, -1]
    gb = np.zeros_like(b[:, 0, :])
    gb[:, -1] = 2.0 * bs / var
    gv = -(bs / var) ** 2
    return gb, gv


def wald_loss(M, XL, y, XR):
    b, var, _ = GLSOracle(M, XL, y).solve(XR)
    return float(np.sum(b[:, 0, -1] ** 2 / var))


def reverse(M, XL, y, XR, gb, gv):
    """(dl/dy, dl/dM) for cotangents gb (m, p) and gv (m,), one trait."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    XL = np.asarray(XL, dtype=np.float64).reshape(n, -1)
    y = np.asarray(y, dtype=np.float64).reshape(n)
    XR = np.asarray(XR, dtype=np.float64)
    Minv = np.linalg.inv(M)
    gy = np.zeros(n)
    Mbar = np.zeros((n, n))
    p = XL.shape[1] + 1
    ep = np.zeros(p)
    ep[-1] = 1.0
    for i, x in enumerate(XR):
        Xi = np.column_stack([XL, x])
        A = Minv @ Xi
        S = Xi.T @ A
        Sinv = np.linalg.inv(S)
        bi = Sinv @ (A.T @ y)
        a = Sinv @ gb[i]
        f = A @ a
        e = Minv @ (y - Xi @ bi)
        t = A @ (Sinv @ ep)
        gy += f
        Mbar -= 0.5 * (np.outer(f, e) + np.outer(e, f))
        Mbar += gv[i] * np.outer(t, t)
    return gy, Mbar


def wald_gradient(Phi, sigma2, h2, XL, y, XR):
    """(loss, dl/dy, dl/dh^2) for l = sum_i b_SNP,i^2 / var_i."""
    M = model_covariance(Phi, sigma2, h2)
    b, var, _ = GLSOracle(M, XL, y).solve(XR)
    gb, gv = wald_loss_cotangents(b, var)
    gy, Mbar = reverse(M, XL, y, XR, gb, gv)
    dM = sigma2 * (Phi - np.eye(Phi.shape[0]))
    return float(np.sum(b[:, 0, -1] ** 2 / var)), gy, float(np.sum(Mbar * dM))


def wald_gradient_contracted(Phi, sigma2, h2, XL, y, XR):
    """wald_gradient without forming dl/dM: the same terms f_i, e_i, t_i,
    evaluated for all SNPs at once with matrix products, and
    <dl/dM, dM> = sum_i (-f_i^T dM e_i + gv_i t_i^T dM t_i) (dM symmetric),
    so that n = 10^4 with a few thousand SNPs runs in seconds."""
    Phi = np.asarray(Phi, dtype=np.float64)
    n = Phi.shape[0]
    M = model_covariance(Phi, sigma2, h2)
    XL = np.asarray(XL, dtype=np.float64).reshape(n, -1)
    y = np.asarray(y, dtype=np.float64).reshape(n)
    XR = np.asarray(XR, dtype=np.float64)
    m, q1 = XR.shape[0], XL.shape[1]
    p = q1 + 1
    Minv = np.linalg.inv(M)
    WL = Minv @ XL                      # M^-1 X_L
    wy = Minv @ y                       # M^-1 y
    WR = Minv @ XR.T                    # column i: M^-1 x_i
    # S_i = X_i^T M^-1 X_i and r_i = X_i^T M^-1 y for every SNP, then b_i
    S = np.empty((m, p, p))
    S[:, :q1, :q1] = XL.T @ WL
    S[:, q1, :q1] = (XR @ WL)
    S[:, :q1, q1] = S[:, q1, :q1]
    S[:, q1, q1] = np.einsum("in,ni->i", XR, WR)
    r = np.empty((m, p))
    r[:, :q1] = XL.T @ wy
    r[:, q1] = XR @ wy
    Sinv = np.linalg.inv(S)
    b = np.einsum("ijk,ik->ij", Sinv, r)
    var = Sinv[:, q1, q1]
    gb, gv = wald_loss_cotangents(b[:, None, :], var)
    a = np.einsum("ijk,ik->ij", Sinv, gb)            # S_i^-1 gb_i
    tau = Sinv[:, :, q1]                             # S_i^-1 e_p
    # f_i = M^-1 X_i a_i, e_i = M^-1 y - M^-1 X_i b_i, t_i = M^-1 X_i tau_i
    F = WL @ a[:, :q1].T + WR * a[:, q1]
    E = wy[:, None] - (WL @ b[:, :q1].T + WR * b[:, q1])
    T = WL @ tau[:, :q1].T + WR * tau[:, q1]
    dM = sigma2 * (Phi - np.eye(n))
    gh2 = float(-np.sum(F * (dM @ E)) + np.sum(gv * np.sum(T * (dM @ T), axis=0)))
    return float(np.sum(b[:, -1] ** 2 / var)), F.sum(axis=1), gh2
