"""Pins for the CPU oracle of Eq. (1): each fixes it against something other
than itself (exact arithmetic, textbook special cases, closed forms and
invariances), so that a dropped term, a wrong sign or index or a transposed
operand in the oracle fails at least one of them.  CPU only."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import GLSOracle, GLSPlain, GLSWhitenedQR, gls_literal
from oracle import gls as oracle_gls
from paper_1304_2272_amd import synth


@pytest.fixture(params=["numpy", "plain_c"])
def Oracle(request):
    """Both oracles meet the same pins: the numpy/LAPACK definition and the
    plain single-threaded C one."""
    return GLSOracle if request.param == "numpy" else GLSPlain


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _spd(n, rng, cond=30.0):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def _problem(n, p, m, seed):
    rng = np.random.default_rng(seed)
    M = _spd(n, rng)
    XL = np.column_stack([np.ones(n), rng.standard_normal((n, p - 2))])
    y = rng.standard_normal(n)
    XR = rng.integers(0, 3, size=(m, n)).astype(np.float64)
    return M, XL, y, XR


# -- P1: exact rational arithmetic -------------------------------------------

def _frac_solve(A, B):
    """Gauss-Jordan over Fractions: A^-1 B exactly (A square, nonsingular)."""
    n = len(A)
    k = len(B[0])
    aug = [list(A[i]) + list(B[i]) for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if aug[r][c] != 0)
        aug[c], aug[piv] = aug[piv], aug[c]
        pv = aug[c][c]
        aug[c] = [v / pv for v in aug[c]]
        for r in range(n):
            if r != c and aug[r][c] != 0:
                f = aug[r][c]
                aug[r] = [vr - f * vc for vr, vc in zip(aug[r], aug[c])]
    return [row[n:n + k] for row in aug]


def _frac_T(A):
    return [list(r) for r in zip(*A)]


def _frac_mm(A, B):
    return [[sum(a * b for a, b in zip(row, col)) for col in zip(*B)] for row in A]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p1_exact_rationals(seed, Oracle):
    rng = np.random.default_rng(100 + seed)
    n, p, m = 7, 3, 4
    A = rng.integers(-3, 4, size=(n, n))
    M = A.T @ A + np.eye(n, dtype=np.int64)          # integer SPD
    XL = np.column_stack([np.ones(n, dtype=np.int64), rng.integers(-4, 5, size=n)])
    y = rng.integers(-9, 10, size=n)
    XR = rng.integers(0, 3, size=(m, n))
    b, var, info = Oracle(M, XL, y).solve(XR)
    Mf = [[Fraction(int(v)) for v in row] for row in M]
    for i in range(m):
        Xi = [[Fraction(int(XL[r, 0])), Fraction(int(XL[r, 1])), Fraction(int(XR[i, r]))] for r in range(n)]
        Af = _frac_solve(Mf, Xi)                      # M^-1 X_i
        N = _frac_mm(_frac_T(Xi), Af)                 # X_i^T M^-1 X_i
        yc = [[Fraction(int(v))] for v in y]
        rhs = _frac_mm(_frac_T(Af), yc)               # X_i^T M^-1 y
        bex = [row[0] for row in _frac_solve(N, rhs)]
        Ninv = _frac_solve(N, [[Fraction(int(r == c)) for c in range(p)] for r in range(p)])
        assert info[i] == 0
        assert _rel(b[i, 0], [float(v) for v in bex]) < 1e-13
        assert abs(var[i] - float(Ninv[p - 1][p - 1])) <= 1e-13 * abs(float(Ninv[p - 1][p - 1]))


# -- P2: explicit inverse by Gauss-Jordan (no factorisation reuse) -----------

def _gauss_jordan_inverse(M):
    n = M.shape[0]
    aug = np.hstack([M.astype(np.float64), np.eye(n)])
    for c in range(n):
        piv = c + int(np.argmax(np.abs(aug[c:, c])))
        aug[[c, piv]] = aug[[piv, c]]
        aug[c] /= aug[c, c]
        for r in range(n):
            if r != c:
                aug[r] -= aug[r, c] * aug[c]
    return aug[:, n:]


def test_p2_explicit_inverse(Oracle):
    M, XL, y, XR = _problem(40, 4, 25, seed=3)
    Minv = _gauss_jordan_inverse(M)
    b, var, _ = Oracle(M, XL, y).solve(XR)
    for i in range(XR.shape[0]):
        Xi = np.column_stack([XL, XR[i]])
        N = Xi.T @ Minv @ Xi
        ref = np.linalg.solve(N, Xi.T @ Minv @ y)
        assert _rel(b[i, 0], ref) < 1e-11
        assert abs(var[i] - np.linalg.inv(N)[-1, -1]) < 1e-11 * abs(var[i])


# -- P3: QR-based GLS through symmetric whitening (Section 2's alternative) --

def test_p3_qr_whitening(Oracle):
    M, XL, y, XR = _problem(60, 5, 20, seed=4)
    w, V = np.linalg.eigh(M)
    Wh = (V / np.sqrt(w)) @ V.T                        # M^{-1/2}, symmetric
    b, _, _ = Oracle(M, XL, y).solve(XR)
    for i in range(XR.shape[0]):
        Xi = np.column_stack([XL, XR[i]])
        Q, R = np.linalg.qr(Wh @ Xi)
        ref = np.linalg.solve(R, Q.T @ (Wh @ y))
        assert _rel(b[i, 0], ref) < 1e-10


# -- P4: planted coefficients, noise-free (fixes bbar_T = X_L^T ybar) -------

@pytest.mark.parametrize("p", [2, 4, 8])
def test_p4_planted_b(p, Oracle):
    prob = synth.make_problem(300, p, seed=11, noise=False)
    XR = synth.snp_block(300, 11, 0, 50)
    beta = prob["beta"][:, 0]
    b, _, info = Oracle(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    assert (info == 0).all()
    want = np.concatenate([beta, [0.0]])
    assert np.max(np.abs(b[:, 0, :] - want)) < 1e-10 * max(1.0, np.max(np.abs(beta)))
    # plant a SNP effect on SNP k
    k, gamma = 17, 0.75
    y2 = prob["Y"][:, 0] + gamma * XR[k]
    b2, _, _ = Oracle(prob["M"], prob["XL"], y2).solve(XR[k:k + 1])
    assert np.max(np.abs(b2[0, 0] - np.concatenate([beta, [gamma]]))) < 1e-10


# -- P5: M = I gives OLS; M = diag(1/w) gives weighted least squares --------

def test_p5_ols_and_wls(Oracle):
    rng = np.random.default_rng(5)
    n, p, m = 80, 4, 12
    XL = np.column_stack([np.ones(n), rng.standard_normal((n, p - 2))])
    y = rng.standard_normal(n)
    XR = rng.integers(0, 3, size=(m, n)).astype(np.float64)
    b, _, _ = Oracle(np.eye(n), XL, y).solve(XR)
    w = rng.uniform(0.2, 5.0, n)
    bw, _, _ = Oracle(np.diag(1.0 / w), XL, y).solve(XR)
    for i in range(m):
        Xi = np.column_stack([XL, XR[i]])
        ref = np.linalg.lstsq(Xi, y, rcond=None)[0]
        assert _rel(b[i, 0], ref) < 1e-12
        sw = np.sqrt(w)
        refw = np.linalg.lstsq(Xi * sw[:, None], y * sw, rcond=None)[0]
        assert _rel(bw[i, 0], refw) < 1e-12


# -- P6: n = p, square invertible X_i: b_i = X_i^-1 y whatever M ------------

def test_p6_square_design(Oracle):
    rng = np.random.default_rng(6)
    n = p = 4
    M = _spd(n, rng, cond=10.0)
    XL = np.column_stack([np.ones(n), rng.standard_normal((n, p - 2))])
    y = rng.standard_normal(n)
    XR = rng.integers(0, 3, size=(6, n)).astype(np.float64)
    b, var, info = Oracle(M, XL, y).solve(XR)
    for i in range(6):
        Xi = np.column_stack([XL, XR[i]])
        if abs(np.linalg.det(Xi)) < 1e-8:
            continue
        Xinv = np.linalg.inv(Xi)
        assert _rel(b[i, 0], Xinv @ y) < 1e-11
        assert abs(var[i] - (Xinv @ M @ Xinv.T)[-1, -1]) < 1e-10 * abs(var[i])


# -- P7: invariances ----------------------------------------------------------

def test_p7_invariances(Oracle):
    M, XL, y, XR = _problem(50, 4, 10, seed=7)
    b, var, _ = Oracle(M, XL, y).solve(XR)
    # scaling M leaves b unchanged (variance scales)
    bs, vs, _ = Oracle(3.5 * M, XL, y).solve(XR)
    assert _rel(bs, b) < 1e-12
    assert _rel(vs, 3.5 * var) < 1e-12
    # consistent permutation of individuals
    perm = np.random.default_rng(8).permutation(50)
    bp, _, _ = Oracle(M[np.ix_(perm, perm)], XL[perm], y[perm]).solve(XR[:, perm])
    assert _rel(bp, b) < 1e-11
    # x -> x + c 1 leaves the SNP coefficient unchanged (intercept absorbs it)
    bc, vc, _ = Oracle(M, XL, y).solve(XR + 2.5)
    assert _rel(bc[:, 0, -1], b[:, 0, -1]) < 1e-10
    assert _rel(vc, var) < 1e-10
    # x -> a x divides it by a
    ba, _, _ = Oracle(M, XL, y).solve(-1.7 * XR)
    assert _rel(ba[:, 0, -1], b[:, 0, -1] / -1.7) < 1e-11
    # duplicate SNP columns give identical results
    bd, _, _ = Oracle(M, XL, y).solve(np.vstack([XR[3], XR[3]]))
    assert np.array_equal(bd[0], bd[1])


# -- P8: Frisch-Waugh-Lovell closed form for the SNP coefficient -------------

def test_p8_fwl_closed_form(Oracle):
    M, XL, y, XR = _problem(70, 6, 15, seed=9)
    Minv = _gauss_jordan_inverse(M)
    P = Minv - Minv @ XL @ np.linalg.inv(XL.T @ Minv @ XL) @ XL.T @ Minv
    b, var, _ = Oracle(M, XL, y).solve(XR)
    for i in range(XR.shape[0]):
        x = XR[i]
        s = x @ P @ x
        assert abs(b[i, 0, -1] - (x @ P @ y) / s) < 1e-10 * max(1.0, abs(b[i, 0, -1]))
        assert abs(var[i] - 1.0 / s) < 1e-10 * var[i]


# -- literal per-SNP form, multiple traits, rank deficiency -------------------

def test_literal_and_traits(Oracle):
    M, XL, _, XR = _problem(30, 3, 8, seed=10)
    Y = np.random.default_rng(12).standard_normal((30, 5))
    b, _, _ = Oracle(M, XL, Y).solve(XR)
    assert b.shape == (8, 5, 3)
    assert _rel(b, gls_literal(M, XL, Y, XR)) < 1e-11
    for j in range(5):
        bj, _, _ = Oracle(M, XL, Y[:, j]).solve(XR)
        assert _rel(b[:, j], bj[:, 0]) < 1e-13


def test_rank_deficient_snp_flagged(Oracle):
    M, XL, y, XR = _problem(40, 4, 5, seed=13)
    XR[2] = 2.0                     # monomorphic: collinear with the intercept
    XR[4] = 0.0                     # all-zero column
    b, var, info = Oracle(M, XL, y).solve(XR)
    assert list(info) == [0, 0, 4, 0, 4]
    assert np.isnan(b[2]).all() and np.isnan(b[4]).all() and np.isnan(var[2])
    assert np.isfinite(b[[0, 1, 3]]).all()


# -- planted mistakes: the pins above must catch them -------------------------

class _YNotWhitened(GLSOracle):
    """Mistake S3 of the printed listing read literally: bbar_T from y, not M^-1 y."""
    def normal_equations(self, XR):
        N, r = super().normal_equations(XR)
        r[:, :self.p - 1, :] = self.XL.T @ self.Y
        return N, r


class _DroppedCross(GLSOracle):
    """A dropped off-diagonal block of X_i^T M^-1 X_i."""
    def normal_equations(self, XR):
        N, r = super().normal_equations(XR)
        N[:, self.p - 1, :self.p - 1] = 0.0
        N[:, :self.p - 1, self.p - 1] = 0.0
        return N, r


class _WrongSign(GLSOracle):
    def normal_equations(self, XR):
        N, r = super().normal_equations(XR)
        r[:, self.p - 1, :] *= -1.0
        return N, r


@pytest.mark.parametrize("bad", [_YNotWhitened, _DroppedCross, _WrongSign])
def test_planted_mistakes_are_caught(bad):
    prob = synth.make_problem(200, 4, seed=21, noise=False)
    XR = synth.snp_block(200, 21, 0, 20)
    beta = prob["beta"][:, 0]
    k, gamma = 5, 0.9
    y = prob["Y"][:, 0] + gamma * XR[k]
    want = np.concatenate([beta, [gamma]])
    good, _, _ = GLSOracle(prob["M"], prob["XL"], y).solve(XR[k:k + 1])
    assert np.max(np.abs(good[0, 0] - want)) < 1e-10
    wrong, _, _ = bad(prob["M"], prob["XL"], y).solve(XR[k:k + 1])
    assert np.max(np.abs(wrong[0, 0] - want)) > 1e-3



# -- the whitened-QR route (Section 2's other OLS solver) ---------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_whitened_qr_exact_rationals(seed):
    # the same integer problems as P1: both routes give the exact b
    rng = np.random.default_rng(100 + seed)
    n, m = 7, 4
    A = rng.integers(-3, 4, size=(n, n))
    M = A.T @ A + np.eye(n, dtype=np.int64)
    XL = np.column_stack([np.ones(n, dtype=np.int64), rng.integers(-4, 5, size=n)])
    y = rng.integers(-9, 10, size=n)
    XR = rng.integers(0, 3, size=(m, n))
    bq, vq, iq = GLSWhitenedQR(M, XL, y).solve(XR)
    Mf = [[Fraction(int(v)) for v in row] for row in M]
    for i in range(m):
        Xi = [[Fraction(int(XL[r, 0])), Fraction(int(XL[r, 1])), Fraction(int(XR[i, r]))] for r in range(n)]
        Af = _frac_solve(Mf, Xi)
        N = _frac_mm(_frac_T(Xi), Af)
        rhs = _frac_mm(_frac_T(Af), [[Fraction(int(v))] for v in y])
        bex = [row[0] for row in _frac_solve(N, rhs)]
        Ninv = _frac_solve(N, [[Fraction(int(r == c)) for c in range(3)] for r in range(3)])
        assert iq[i] == 0
        assert _rel(bq[i, 0], [float(v) for v in bex]) < 1e-13
        assert abs(vq[i] - float(Ninv[2][2])) <= 1e-13 * abs(float(Ninv[2][2]))


def test_whitened_qr_planted_ols_traits_and_rank():
    prob = synth.make_problem(300, 4, seed=11, noise=False)
    XR = synth.snp_block(300, 11, 0, 30)
    b, _, info = GLSWhitenedQR(prob["M"], prob["XL"], prob["Y"]).solve(XR)
    assert (info == 0).all()
    want = np.concatenate([prob["beta"][:, 0], [0.0]])
    assert np.max(np.abs(b[:, 0, :] - want)) < 1e-10
    # M = I: ordinary least squares
    rng = np.random.default_rng(5)
    n = 80
    XL = np.column_stack([np.ones(n), rng.standard_normal((n, 2))])
    Y = rng.standard_normal((n, 3))
    XR = rng.integers(0, 3, size=(6, n)).astype(np.float64)
    b, _, _ = GLSWhitenedQR(np.eye(n), XL, Y).solve(XR)
    for i in range(6):
        ref = np.linalg.lstsq(np.column_stack([XL, XR[i]]), Y, rcond=None)[0]
        assert _rel(b[i], ref.T) < 1e-12
    # rank-deficient SNPs flagged as by the plain route
    M, XL, y, XR = _problem(40, 4, 5, seed=13)
    XR[2] = 2.0
    XR[4] = 0.0
    b, var, info = GLSWhitenedQR(M, XL, y).solve(XR)
    assert list(info) == [0, 0, 4, 0, 4] and np.isnan(b[2]).all() and np.isnan(var[4])
    bo, vo, _ = GLSOracle(M, XL, y).solve(XR)
    assert _rel(b[[0, 1, 3]], bo[[0, 1, 3]]) < 1e-11 and _rel(var[[0, 1, 3]], vo[[0, 1, 3]]) < 1e-11


def _refined_reference(M, XL, y, XR):
    """b_SNP and var of Eq. (1) to near extended precision: M^-1 [x | X_L | y]
    by float64 LU with three steps of iterative refinement whose residuals
    are formed in long double, then the p x p normal equations in long
    double (Gauss-Jordan)."""
    import scipy.linalg as sla
    m, n = XR.shape
    p = XL.shape[1] + 1
    R = np.concatenate([XR.T, XL, y[:, None]], axis=1)
    lu = sla.lu_factor(M)
    A = sla.lu_solve(lu, R).astype(np.longdouble)
    Ml, Rl = M.astype(np.longdouble), R.astype(np.longdouble)
    for _ in range(3):
        A = A + sla.lu_solve(lu, (Rl - Ml @ A).astype(np.float64)).astype(np.longdouble)
    bs = np.empty(m)
    vs = np.empty(m)
    for i in range(m):
        cols = list(range(m, m + p - 1)) + [i]
        N = Rl[:, cols].T @ A[:, cols]
        r = A[:, cols].T @ Rl[:, -1]
        aug = np.concatenate([N, r[:, None], np.eye(p, dtype=np.longdouble)], axis=1)
        for k in range(p):
            aug[k] = aug[k] / aug[k, k]
            for j in range(p):
                if j != k:
                    aug[j] = aug[j] - aug[j, k] * aug[k]
        bs[i] = float(aug[p - 1, p])
        vs[i] = float(aug[p - 1, 2 * p])
    return bs, vs


def test_whitened_qr_keeps_snp_digits_at_high_condition():
    # h^2 = 0.9999 with Phi of rank 60 < n: kappa(M) about 1e5.  Against an
    # extended-precision solution the whitened QR route's SNP coefficients in
    # standard-error units are within a few kappa(M) u (the forward error of a
    # backward-stable solve), while the plain route's X_i^T M^-1 X_i loses
    # about a hundred times more (printed)
    n, p, m, seed = 400, 4, 40, 31
    prob = synth.make_problem(n, p, seed, h2=0.9999, k=60)
    M, XL, y = prob["M"], prob["XL"], prob["Y"][:, 0]
    XR = synth.snp_block(n, seed, 0, m)
    ev = np.linalg.eigvalsh(M)
    assert ev[-1] / ev[0] > 1e4
    bs, vs = _refined_reference(M, XL, y, XR)
    bq, vq, _ = GLSWhitenedQR(M, XL, y).solve(XR)
    bo, vo, _ = GLSOracle(M, XL, y).solve(XR)
    se_q = np.max(np.abs(bq[:, 0, -1] - bs) / np.sqrt(vs))
    se_o = np.max(np.abs(bo[:, 0, -1] - bs) / np.sqrt(vs))
    print(f"kappa(M) {ev[-1] / ev[0]:.3g}: SE error whitened QR {se_q:.3e}, normal equations {se_o:.3e}")
    kappa = ev[-1] / ev[0]
    assert se_q < 4.0 * kappa * 2.0 ** -53
    assert _rel(vq, vs) < 1e-11 and _rel(vo, vs) < 1e-9


# -- the two oracles against each other on random shapes ----------------------

@pytest.mark.parametrize("seed", range(6))
def test_plain_c_oracle_matches_numpy_oracle(seed):
    # two implementations of Eq. (1) that share nothing but the definition
    # (LU with LAPACK against a hand-written Cholesky and elimination)
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(5, 400))
    p = int(rng.integers(2, min(12, n) + 1))
    m = int(rng.integers(1, 60))
    t = int(rng.integers(1, 4))
    M, XL, _, XR = _problem(n, p, m, seed=900 + seed)
    Y = rng.standard_normal((n, t))
    b0, v0, i0 = GLSOracle(M, XL, Y).solve(XR)
    b1, v1, i1 = GLSPlain(M, XL, Y).solve(XR)
    assert np.array_equal(i0, i1)
    ok = i0 == 0
    assert _rel(b1[ok], b0[ok]) < 1e-10 and _rel(v1[ok], v0[ok]) < 1e-10


def test_plain_c_oracle_refuses_a_non_spd_m():
    M, XL, y, _ = _problem(20, 3, 1, seed=31)
    M = M.copy()
    M[7, 7] = -1.0
    with pytest.raises(np.linalg.LinAlgError):
        GLSPlain(M, XL, y)
