/*
 * Plain single-threaded float64 reference of the GLS solves of Eq. (1):
 *
 *     b_i = (X_i^T M^-1 X_i)^-1 X_i^T M^-1 y,    X_i = [X_L | x_i],  i = 1..m.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the entry module's smoke check and the
 * benchmark's CPU baseline load it; the GPU library never links it and it
 * shares no code with it.  No BLAS, no threads, no fast-math: every loop is
 * written out here.
 *
 * Steps (the plain definition, with M^-1 applied through a Cholesky factor
 * M = L L^T of the lower triangle, Section 2):
 *   set-up   L by an unblocked left-looking Cholesky; A_L = M^-1 X_L and
 *            A_y = M^-1 y by forward then backward substitution; the SNP-free
 *            parts of the normal equations, X_L^T A_L and A_L^T y.
 *   per SNP  a = M^-1 x_i (two substitutions, 2 n^2 flops); the p x p normal
 *            equations N_i = X_i^T M^-1 X_i and r_i = X_i^T M^-1 y, their
 *            last row (and, M being symmetric, last column) x_i^T [A_L | a]
 *            and x_i^T A_y;
 *            N_i [b_i | v] = [r_i | e_p] by Gaussian elimination with partial
 *            pivoting; var_i = v_p = [N_i^-1]_pp.
 * A SNP whose Schur complement s_i = 1 / var_i falls to or below rank_tol
 * times (N_i)_pp (X_i numerically rank deficient) gets info_i = p and NaN
 * b_i and var_i.
 *
 * Layouts: M column-major n x n (only the lower triangle is read), X_L
 * column-major n x (p-1), Y column-major n x t, XR SNP-major (SNP i at
 * XR + i * ldx), b as (m, t, p) row-major, all float64.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* doubles of the set-up workspace */
int64_t gls_plain_work_size(int64_t n, int p, int t) {
    const int64_t q = p - 1;
    return n * n + n * q + n * t + q * q + q * t;
}

/* L z = v (forward), L lower triangular column-major */
static void forward(const double* L, int64_t n, double* v) {
    for (int64_t j = 0; j < n; ++j) {
        const double* col = L + j * n;
        const double z = v[j] / col[j];
        v[j] = z;
        for (int64_t i = j + 1; i < n; ++i) v[i] -= col[i] * z;
    }
}

/* L^T w = v (backward) */
static void backward(const double* L, int64_t n, double* v) {
    for (int64_t j = n - 1; j >= 0; --j) {
        const double* col = L + j * n;
        double s = v[j];
        for (int64_t i = j + 1; i < n; ++i) s -= col[i] * v[i];
        v[j] = s / col[j];
    }
}

/* Set-up.  Returns 0, or the 1-based order of the first non-positive pivot
 * of M, or -1 for bad sizes. */
int64_t gls_plain_setup(int64_t n, int p, int t, const double* M, int64_t ldm, const double* XL, int64_t ldxl,
                        const double* Y, int64_t ldy, double* work) {
    if (n < 1 || p < 2 || t < 1 || ldm < n || ldxl < n || ldy < n) return -1;
    const int64_t q = p - 1;
    double* L = work;
    double* AL = L + n * n;
    double* Ay = AL + n * q;
    double* NLL = Ay + n * t;
    double* rL = NLL + q * q;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) L[i + j * n] = i >= j ? M[i + j * ldm] : 0.0;
    /* left-looking Cholesky: column j of L from the columns before it */
    for (int64_t j = 0; j < n; ++j) {
        double* cj = L + j * n;
        for (int64_t k = 0; k < j; ++k) {
            const double* ck = L + k * n;
            const double ljk = ck[j];
            if (ljk == 0.0) continue;
            for (int64_t i = j; i < n; ++i) cj[i] -= ck[i] * ljk;
        }
        if (!(cj[j] > 0.0)) return j + 1;
        const double d = sqrt(cj[j]);
        cj[j] = d;
        for (int64_t i = j + 1; i < n; ++i) cj[i] /= d;
    }
    for (int64_t c = 0; c < q; ++c) {
        double* a = AL + c * n;
        memcpy(a, XL + c * ldxl, (size_t)n * sizeof(double));
        forward(L, n, a);
        backward(L, n, a);
    }
    for (int64_t c = 0; c < t; ++c) {
        double* a = Ay + c * n;
        memcpy(a, Y + c * ldy, (size_t)n * sizeof(double));
        forward(L, n, a);
        backward(L, n, a);
    }
    for (int64_t r = 0; r < q; ++r)
        for (int64_t c = 0; c < q; ++c) {
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) s += XL[i + r * ldxl] * AL[i + c * n];
            NLL[r * q + c] = s;
        }
    for (int64_t r = 0; r < q; ++r)
        for (int64_t c = 0; c < t; ++c) {
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) s += AL[i + r * n] * Y[i + c * ldy];
            rL[r * t + c] = s;
        }
    return 0;
}

/* N x = B for a p x p N (row-major, destroyed) and k right-hand sides
 * (row-major p x k, overwritten with x); Gaussian elimination with partial
 * pivoting.  Returns 0, or 1 for a zero pivot. */
static int ge_solve(double* N, int p, double* B, int k) {
    for (int c = 0; c < p; ++c) {
        int piv = c;
        for (int r = c + 1; r < p; ++r)
            if (fabs(N[r * p + c]) > fabs(N[piv * p + c])) piv = r;
        if (N[piv * p + c] == 0.0) return 1;
        if (piv != c) {
            for (int j = 0; j < p; ++j) {
                const double s = N[c * p + j]; N[c * p + j] = N[piv * p + j]; N[piv * p + j] = s;
            }
            for (int j = 0; j < k; ++j) {
                const double s = B[c * k + j]; B[c * k + j] = B[piv * k + j]; B[piv * k + j] = s;
            }
        }
        for (int r = c + 1; r < p; ++r) {
            const double f = N[r * p + c] / N[c * p + c];
            for (int j = c; j < p; ++j) N[r * p + j] -= f * N[c * p + j];
            for (int j = 0; j < k; ++j) B[r * k + j] -= f * B[c * k + j];
        }
    }
    for (int c = p - 1; c >= 0; --c)
        for (int j = 0; j < k; ++j) {
            double s = B[c * k + j];
            for (int i = c + 1; i < p; ++i) s -= N[c * p + i] * B[i * k + j];
            B[c * k + j] = s / N[c * p + c];
        }
    return 0;
}

/* m SNPs.  tmp: n doubles.  p <= 64, t <= 256. */
int gls_plain_solve(const double* work, int64_t n, int p, int t, int64_t m, const double* XR, int64_t ldx,
                    double* b, double* var, int32_t* info, double rank_tol, double* tmp) {
    if (n < 1 || p < 2 || p > 64 || t < 1 || t > 256 || m < 0 || ldx < n) return -1;
    const int64_t q = p - 1;
    const double* L = work;
    const double* AL = L + n * n;
    const double* Ay = AL + n * q;
    const double* NLL = Ay + n * t;
    const double* rL = NLL + q * q;
    double N[64 * 64], B[64 * 257];
    const int k = t + 1;
    for (int64_t i = 0; i < m; ++i) {
        const double* x = XR + i * ldx;
        memcpy(tmp, x, (size_t)n * sizeof(double));
        forward(L, n, tmp);
        backward(L, n, tmp);                       /* tmp = M^-1 x_i */
        for (int64_t r = 0; r < q; ++r)
            for (int64_t c = 0; c < q; ++c) N[r * p + c] = NLL[r * q + c];
        /* x_i^T M^-1 X_L, the last row and (M symmetric) the last column */
        for (int64_t c = 0; c < q; ++c) {
            double s = 0.0;
            for (int64_t e = 0; e < n; ++e) s += x[e] * AL[e + c * n];
            N[q * p + c] = s;
            N[c * p + q] = s;
        }
        {
            double s = 0.0;                        /* x_i^T M^-1 x_i */
            for (int64_t e = 0; e < n; ++e) s += x[e] * tmp[e];
            N[q * p + q] = s;
        }
        for (int64_t r = 0; r < q; ++r)
            for (int c = 0; c < t; ++c) B[r * k + c] = rL[r * t + c];
        for (int c = 0; c < t; ++c) {
            double s = 0.0;                        /* x_i^T M^-1 y */
            for (int64_t e = 0; e < n; ++e) s += x[e] * Ay[e + c * n];
            B[q * k + c] = s;
        }
        for (int r = 0; r < p; ++r) B[r * k + t] = r == q ? 1.0 : 0.0;
        const double npp = N[q * p + q];
        const int singular = ge_solve(N, p, B, k);
        const double v = singular ? NAN : B[q * k + t];
        const double s = 1.0 / v;
        if (singular || !isfinite(v) || !(s > rank_tol * npp)) {
            if (info) info[i] = p;
            for (int c = 0; c < t; ++c)
                for (int r = 0; r < p; ++r) b[(i * t + c) * p + r] = NAN;
            if (var) var[i] = NAN;
            continue;
        }
        if (info) info[i] = 0;
        for (int c = 0; c < t; ++c)
            for (int r = 0; r < p; ++r) b[(i * t + c) * p + r] = B[r * k + c];
        if (var) var[i] = v;
    }
    return 0;
}
