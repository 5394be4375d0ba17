"""CPU oracle for the m generalized least-squares solves of Eq. (1).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module: only the tests, the smoke check of the entry module and the
CPU-baseline leg of the benchmark use it.  It shares no code with the GPU
library.

What it computes is the plain definition of Eq. (1) (Section 1):

    b_i = (X_i^T M^-1 X_i)^-1 X_i^T M^-1 y,   X_i = [X_L | x_i],  i = 1..m,

in float64, with each X_i formed explicitly and its p x p normal equations
solved directly (Section 2: the OLS form S_i b_i = bbar_i solved through the
normal equations).  M^-1 is applied through an LU factorisation with partial
pivoting of M (a LAPACK primitive), deliberately not the Cholesky factor the
paper's restructuring (Algorithms 1 and 2) is built on.  The only reuse is that
one factorisation of M serves every right-hand side.

Besides b_i it reports var_i = [(X_i^T M^-1 X_i)^-1]_{pp}, the variance of the
SNP coefficient (M is the covariance of y, so this p x p inverse is Cov(b_i);
the footnote of Section 3 mentions that a p x p symmetric matrix accompanies
each b_i), and info_i = p when X_i is numerically rank deficient (the problem
statement assumes full rank; this is the reading adopted for the degenerate
case): the Schur complement s_i = 1 / var_i falls to or below ``rank_tol``
times the (p,p) entry of X_i^T M^-1 X_i.  Rank-deficient SNPs get NaN b_i.

Multiple traits (columns of y) share M and X_i: b has shape (m, t, p).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

RANK_TOL = 1e-10


def _as_2d(Y):
    Y = np.asarray(Y, dtype=np.float64)
    return Y[:, None] if Y.ndim == 1 else Y


class GLSOracle:
    """Plain Eq. (1) solver: factor M once (LU), then per-SNP normal equations."""

    def __init__(self, M, XL, Y, rank_tol: float = RANK_TOL):
        M = np.asarray(M, dtype=np.float64)
        self.n = M.shape[0]
        self.XL = np.asarray(XL, dtype=np.float64).reshape(self.n, -1)
        self.Y = _as_2d(Y)
        self.p = self.XL.shape[1] + 1
        self.t = self.Y.shape[1]
        self.rank_tol = rank_tol
        self._lu = sla.lu_factor(M, check_finite=True)
        # M^-1 X_L and M^-1 y: the columns of M^-1 X_i that do not depend on i
        self.MinvXL = sla.lu_solve(self._lu, self.XL)
        self.MinvY = sla.lu_solve(self._lu, self.Y)

    def minv(self, B):
        """M^-1 B for an n x k right-hand side."""
        return sla.lu_solve(self._lu, np.asarray(B, dtype=np.float64))

    def normal_equations(self, XR):
        """N_i = X_i^T M^-1 X_i (m,p,p) and r_i = X_i^T M^-1 y (m,p,t)."""
        XR = np.asarray(XR, dtype=np.float64)          # (m, n) SNP-major
        m, p = XR.shape[0], self.p
        A = self.minv(XR.T)                              # n x m, column i = M^-1 x_i
        N = np.empty((m, p, p))
        N[:, :p - 1, :p - 1] = self.XL.T @ self.MinvXL
        N[:, p - 1, :p - 1] = XR @ self.MinvXL           # x_i^T M^-1 X_L
        N[:, :p - 1, p - 1] = (self.XL.T @ A).T          # X_L^T M^-1 x_i
        N[:, p - 1, p - 1] = np.einsum("in,ni->i", XR, A)
        r = np.empty((m, p, self.t))
        r[:, :p - 1, :] = self.MinvXL.T @ self.Y
        r[:, p - 1, :] = A.T @ self.Y                    # x_i^T M^-1 y
        return N, r

    def solve(self, XR):
        """b (m,t,p), var (m,), info (m,) int32 for SNP-major dosages XR (m,n)."""
        N, r = self.normal_equations(XR)
        return solve_normal_equations(N, r, self.rank_tol)


class GLSWhitenedQR:
    """Eq. (1) through the reduction of Section 2 with its other OLS solver.

    Section 2 turns each GLS problem into ordinary least squares by whitening
    with a factor of M (M = L L^T, Xbar_i = L^-1 X_i, ybar = L^-1 y) and names
    QR as the alternative to the normal equations for the OLS step.  This
    class does exactly that: a Cholesky factor of M and triangular solves
    (LAPACK primitives) for the whitening, then Householder QR of every
    whitened Xbar_i = [Xbar_L | xbar_i] (numpy), b_i = R^-1 Q^T ybar and
    var_i = [(Xbar_i^T Xbar_i)^-1]_pp = 1 / R_pp^2.  It forms no M^-1 X_i and
    no normal equations, so where M is ill-conditioned its SNP coefficients
    keep far more digits than those of GLSOracle (whose X_i^T M^-1 X_i loses
    about kappa(M) u): it serves as the reference of the SNP coefficient in
    standard-error units there.  info_i = p when R_pp^2 falls to or below
    rank_tol * ||xbar_i||^2 (the Schur complement s_i against S_BR, as in
    GLSOracle).
    """

    def __init__(self, M, XL, Y, rank_tol: float = RANK_TOL):
        M = np.asarray(M, dtype=np.float64)
        self.n = M.shape[0]
        XL = np.asarray(XL, dtype=np.float64).reshape(self.n, -1)
        self.p = XL.shape[1] + 1
        self.rank_tol = rank_tol
        self._L = sla.cholesky(M, lower=True, check_finite=True)
        self.XLb = sla.solve_triangular(self._L, XL, lower=True)
        self.Yb = sla.solve_triangular(self._L, _as_2d(Y), lower=True)

    def solve(self, XR):
        """b (m,t,p), var (m,), info (m,) int32 for SNP-major dosages XR (m,n)."""
        XR = np.asarray(XR, dtype=np.float64)
        m, p, t = XR.shape[0], self.p, self.Yb.shape[1]
        b = np.full((m, t, p), np.nan)
        var = np.full(m, np.nan)
        info = np.zeros(m, dtype=np.int32)
        Zb = sla.solve_triangular(self._L, XR.T, lower=True)        # n x m
        for i in range(m):
            Xb = np.column_stack([self.XLb, Zb[:, i]])
            Q, R = np.linalg.qr(Xb)
            rpp2 = R[p - 1, p - 1] ** 2
            if not rpp2 > self.rank_tol * float(Zb[:, i] @ Zb[:, i]):
                info[i] = p
                continue
            b[i] = sla.solve_triangular(R, Q.T @ self.Yb).T
            var[i] = 1.0 / rpp2
        return b, var, info


def solve_normal_equations(N, r, rank_tol: float = RANK_TOL):
    """Solve N_i b_i = r_i per SNP (LU with pivoting), with var_i and info_i."""
    m, p, _ = N.shape
    t = r.shape[2]
    b = np.full((m, t, p), np.nan)
    var = np.full(m, np.nan)
    info = np.zeros(m, dtype=np.int32)
    if m == 0:
        return b, var, info
    try:
        Ninv = np.linalg.inv(N)
        ok = np.ones(m, dtype=bool)
    except np.linalg.LinAlgError:
        Ninv = np.full_like(N, np.nan)
        ok = np.zeros(m, dtype=bool)
        for i in range(m):
            try:
                Ninv[i] = np.linalg.inv(N[i])
                ok[i] = True
            except np.linalg.LinAlgError:
                pass
    v = Ninv[:, p - 1, p - 1]
    with np.errstate(divide="ignore", invalid="ignore"):
        s = 1.0 / v
        good = ok & np.isfinite(v) & (s > rank_tol * N[:, p - 1, p - 1])
    info[~good] = p
    if good.any():
        b[good] = np.swapaxes(np.linalg.solve(N[good], r[good]), 1, 2)
        var[good] = v[good]
    return b, var, info


def gls_literal(M, XL, Y, XR):
    """Eq. (1) written out with no reuse at all: one dense solve with M per SNP.

    Only for tiny inputs (it costs O(n^3) per SNP).  Returns b (m,t,p).
    """
    M = np.asarray(M, dtype=np.float64)
    XL = np.asarray(XL, dtype=np.float64).reshape(M.shape[0], -1)
    Y = _as_2d(Y)
    XR = np.asarray(XR, dtype=np.float64)
    out = []
    for x in XR:
        Xi = np.column_stack([XL, x])
        A = np.linalg.solve(M, Xi)
        out.append(np.linalg.solve(Xi.T @ A, A.T @ Y).T)
    return np.array(out)
