// Per-SNP kernels of the per-block hot path (Algorithm 2, loop body) and of
// its reverse pass:
//   snp_cross_w     x^T W with W = M^-1 [X_L | y] (reduced-precision paths);
//   partial_chunks  the triangular product's partial sums reduced in chunks;
//   snp_solve       per-SNP p x p Cholesky solve (Algorithm 1, last two lines
//                   of the loop) with optional float64 refinement;
//   snp_backward, sum_columns, dosage_gemv   the reverse pass.
#include "internal.h"

#include <math.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

namespace gwas {
namespace {

// x_j^T W[:, q]: each wave takes 8 SNP columns, lanes stride over k.
constexpr int XW_COLS = 8;
constexpr int XW_Q = 8;
template <typename XT>
__global__ __launch_bounds__(256) void snp_cross_w_kernel(const XT* __restrict__ X, int64_t ldx,
                                                          int64_t n, int64_t cols,
                                                          const double* __restrict__ W, int64_t ldw,
                                                          int Qc, double* __restrict__ xw,
                                                          int64_t ldxw) {
    const int lane = threadIdx.x & 63;
    const int64_t colbase = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * XW_COLS;
    if (colbase >= cols) return;
    for (int q0 = 0; q0 < Qc; q0 += XW_Q) {
        double s[XW_COLS][XW_Q];
#pragma unroll
        for (int c = 0; c < XW_COLS; ++c)
#pragma unroll
            for (int q = 0; q < XW_Q; ++q) s[c][q] = 0.0;
        for (int64_t k = lane; k < n; k += 64) {
            double w[XW_Q];
#pragma unroll
            for (int q = 0; q < XW_Q; ++q) w[q] = (q0 + q < Qc) ? W[k + (q0 + q) * ldw] : 0.0;
#pragma unroll
            for (int c = 0; c < XW_COLS; ++c) {
                const int64_t col = colbase + c;
                const double x = (col < cols) ? (double)X[col * ldx + k] : 0.0;
#pragma unroll
                for (int q = 0; q < XW_Q; ++q) s[c][q] += x * w[q];
            }
        }
#pragma unroll
        for (int c = 0; c < XW_COLS; ++c)
#pragma unroll
            for (int q = 0; q < XW_Q; ++q) {
                double v = s[c][q];
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
                const int64_t col = colbase + c;
                if (lane == 0 && col < cols && q0 + q < Qc) xw[(q0 + q) * ldxw + col] = v;
            }
    }
}

// One thread per SNP.  With R = chol(S_TL) fixed, the Cholesky factor of
// S_i = [[S_TL, S_BL^T], [S_BL, S_BR]] is [[R, 0], [u^T, sqrt(s)]] with
// u = R^-1 S_BL^T and s = S_BR - u^T u, so b_i follows from two triangular
// solves with R and one division by s.  Optional float64 refinement steps
// b <- b + S_i^-1 (bbar_i - S_i b) reuse the same factor.
template <int Q1>
__global__ __launch_bounds__(128) void snp_solve_kernel(SolveArgs a) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.cols) return;
    const int t = a.t;
    const double* R = a.consts + consts_R(Q1);
    const double* V = a.consts + consts_v(Q1);
    const double* STL = a.consts + consts_STL(Q1, t);
    const double* BT = a.consts + consts_bT(Q1, t);

    double sbl[Q1];
    double sbr = 0.0;
#pragma unroll
    for (int q = 0; q < Q1; ++q) sbl[q] = 0.0;
    for (int64_t pb = 0; pb < a.npb; ++pb) {
        const double* P = a.part + pb * a.Q * a.ldp + j;
        if (!a.xw) {
#pragma unroll
            for (int q = 0; q < Q1; ++q) sbl[q] += P[q * a.ldp];
        }
        sbr += P[(a.Q - 1) * a.ldp];
    }
    if (a.xw) {
#pragma unroll
        for (int q = 0; q < Q1; ++q) sbl[q] = a.xw[q * a.ldxw + j];
    }
    double u[Q1];
#pragma unroll
    for (int r = 0; r < Q1; ++r) {
        double s = sbl[r];
#pragma unroll
        for (int k = 0; k < r; ++k) s -= R[r + k * Q1] * u[k];
        u[r] = s / R[r + r * Q1];
    }
    double s = sbr;
#pragma unroll
    for (int r = 0; r < Q1; ++r) s -= u[r] * u[r];
    const bool ok = (s > a.rank_tol * sbr) && isfinite(s) && isfinite(sbr);
    const double nan = __builtin_nan("");
    if (a.var) a.var[j] = ok ? 1.0 / s : nan;
    if (a.info) a.info[j] = ok ? 0 : Q1 + 1;
    double* bj = a.b + j * a.ldb;
    for (int jt = 0; jt < t; ++jt) {
        double bB;
        if (a.xw) {
            bB = a.xw[(Q1 + jt) * a.ldxw + j];
        } else {
            bB = 0.0;
            for (int64_t pb = 0; pb < a.npb; ++pb) bB += a.part[(pb * a.Q + Q1 + jt) * a.ldp + j];
        }
        if (!ok) {
            for (int r = 0; r <= Q1; ++r) bj[jt * (Q1 + 1) + r] = nan;
            continue;
        }
        const double* v = V + jt * Q1;
        double c = bB;
#pragma unroll
        for (int r = 0; r < Q1; ++r) c -= u[r] * v[r];
        double bs = c / s;
        double bl[Q1];
        // R^T bl = v - u bs
#pragma unroll
        for (int r = Q1 - 1; r >= 0; --r) {
            double w = v[r] - u[r] * bs;
#pragma unroll
            for (int k = r + 1; k < Q1; ++k) w -= R[k + r * Q1] * bl[k];
            bl[r] = w / R[r + r * Q1];
        }
        for (int it = 0; it < a.refine; ++it) {
            // residual of S_i b = bbar_i in float64
            double rt[Q1];
#pragma unroll
            for (int r = 0; r < Q1; ++r) {
                double acc = BT[r + jt * Q1] - sbl[r] * bs;
#pragma unroll
                for (int k = 0; k < Q1; ++k) acc -= STL[r + k * Q1] * bl[k];
                rt[r] = acc;
            }
            double rb = bB - sbr * bs;
#pragma unroll
            for (int k = 0; k < Q1; ++k) rb -= sbl[k] * bl[k];
            // solve with the factor: y = R^-1 rt, dB = (rb - u.y)/s, dT = R^-T (y - u dB)
            double y[Q1];
#pragma unroll
            for (int r = 0; r < Q1; ++r) {
                double w = rt[r];
#pragma unroll
                for (int k = 0; k < r; ++k) w -= R[r + k * Q1] * y[k];
                y[r] = w / R[r + r * Q1];
            }
            double dB = rb;
#pragma unroll
            for (int r = 0; r < Q1; ++r) dB -= u[r] * y[r];
            dB /= s;
            double dT[Q1];
#pragma unroll
            for (int r = Q1 - 1; r >= 0; --r) {
                double w = y[r] - u[r] * dB;
#pragma unroll
                for (int k = r + 1; k < Q1; ++k) w -= R[k + r * Q1] * dT[k];
                dT[r] = w / R[r + r * Q1];
            }
#pragma unroll
            for (int r = 0; r < Q1; ++r) bl[r] += dT[r];
            bs += dB;
        }
#pragma unroll
        for (int r = 0; r < Q1; ++r) bj[jt * (Q1 + 1) + r] = bl[r];
        bj[jt * (Q1 + 1) + Q1] = bs;
    }
}

// Reverse pass through the per-SNP solves, one SNP per thread (one trait).
// The factor of S = [[S_TL, S_BL^T], [S_BL, S_BR]] is [[R, 0], [u^T, sqrt(s)]]
// with u = R^-1 S_BL^T and s = 1/var; S^-1 v follows from two solves with it.
template <int Q1>
__global__ __launch_bounds__(128) void snp_backward_kernel(BackArgs a) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.cols) return;
    constexpr int P = Q1 + 1;
    double* out = a.contrib + j;
    if (a.info[j] != 0) {
        for (int k = 0; k <= P; ++k) out[k * a.ldc] = 0.0;
        a.coef[j] = 0.0;
        return;
    }
    const double* R = a.consts + consts_R(Q1);
    double sbl[Q1], h[Q1];
    double eta = 0.0, hy = 0.0;
#pragma unroll
    for (int q = 0; q < Q1; ++q) {
        sbl[q] = a.xw[q * a.ldxw + j];
        h[q] = 0.0;
    }
    for (int64_t pb = 0; pb < a.npb; ++pb) {
        const double* Pp = a.part + pb * (P + 1) * a.ldp + j;
#pragma unroll
        for (int q = 0; q < Q1; ++q) h[q] += Pp[q * a.ldp];       // w^T W_L
        hy += Pp[Q1 * a.ldp];                                       // w^T w_y
        eta += Pp[P * a.ldp];                                       // w^T w
    }
    const double xwy = a.xw[Q1 * a.ldxw + j];                       // x^T w_y
    const double var = a.var[j];
    const double s = 1.0 / var;
    double u[Q1];
#pragma unroll
    for (int r = 0; r < Q1; ++r) {
        double t = sbl[r];
#pragma unroll
        for (int k = 0; k < r; ++k) t -= R[r + k * Q1] * u[k];
        u[r] = t / R[r + r * Q1];
    }
    // v = S^-1 g for a p-vector g (last entry g[Q1])
    auto solve = [&](const double (&g)[P], double (&v)[P]) {
        double y[Q1];
#pragma unroll
        for (int r = 0; r < Q1; ++r) {
            double t = g[r];
#pragma unroll
            for (int k = 0; k < r; ++k) t -= R[r + k * Q1] * y[k];
            y[r] = t / R[r + r * Q1];
        }
        double yb = g[Q1];
#pragma unroll
        for (int r = 0; r < Q1; ++r) yb -= u[r] * y[r];
        const double vb = yb / s;
#pragma unroll
        for (int r = Q1 - 1; r >= 0; --r) {
            double t = y[r] - u[r] * vb;
#pragma unroll
            for (int k = r + 1; k < Q1; ++k) t -= R[k + r * Q1] * v[k];
            v[r] = t / R[r + r * Q1];
        }
        v[Q1] = vb;
    };
    double g[P], av[P], tau[P], e[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        g[k] = a.gb[j * a.ldgb + k];
        e[k] = (k == Q1) ? 1.0 : 0.0;
    }
    solve(g, av);
    solve(e, tau);
    const double gv = a.gv ? a.gv[j] : 0.0;
    // Q = [[G, h], [h^T, eta]], q = [gy0; hy]
    double bb[P];
#pragma unroll
    for (int k = 0; k < P; ++k) bb[k] = a.b[j * a.ldb + k];
    auto Qmul = [&](const double (&x)[P], double (&y)[P]) {
#pragma unroll
        for (int r = 0; r < Q1; ++r) {
            double t = h[r] * x[Q1];
#pragma unroll
            for (int k = 0; k < Q1; ++k) t += a.G[r + k * Q1] * x[k];
            y[r] = t;
        }
        double t = eta * x[Q1];
#pragma unroll
        for (int k = 0; k < Q1; ++k) t += h[k] * x[k];
        y[Q1] = t;
    };
    double Qb[P], Qt[P];
    Qmul(bb, Qb);
    Qmul(tau, Qt);
    double tr = 0.0, tqt = 0.0;
#pragma unroll
    for (int k = 0; k < Q1; ++k) tr -= av[k] * (a.gy0[k] - Qb[k]);
    tr -= av[Q1] * (hy - Qb[Q1]);
#pragma unroll
    for (int k = 0; k < P; ++k) tqt += tau[k] * Qt[k];
    tr += gv * tqt;
#pragma unroll
    for (int k = 0; k < Q1; ++k) out[k * a.ldc] = av[k];
    out[Q1 * a.ldc] = tr;
    out[P * a.ldc] = gv * var;
    a.coef[j] = av[Q1];
    (void)xwy;
}

// out[(g * Q + q) * ldo + j] = sum of part[(pb * Q + q) * ldp + j] over the
// chunk pb in [g * chunk, min((g + 1) * chunk, npb)), in ascending pb: one
// thread per (chunk, row, SNP), SNP fastest for coalesced loads.
__global__ __launch_bounds__(256) void partial_chunks_kernel(const double* __restrict__ part, int64_t ldp,
                                                             int64_t npb, int Q, int64_t cols, int chunk,
                                                             int64_t G, double* __restrict__ out,
                                                             int64_t ldo) {
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= cols * Q * G) return;
    const int64_t j = id % cols;
    const int64_t q = (id / cols) % Q;
    const int64_t g = id / (cols * Q);
    const int64_t pb1 = std::min<int64_t>(npb, (g + 1) * chunk);
    double acc = 0.0;
    for (int64_t pb = g * chunk; pb < pb1; ++pb) acc += part[(pb * Q + q) * ldp + j];
    out[(g * Q + q) * ldo + j] = acc;
}

__global__ __launch_bounds__(256) void sum_columns_kernel(const double* __restrict__ c, int64_t ldc,
                                                          int64_t cols, double* __restrict__ acc) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    double t = 0.0;
    for (int64_t j = threadIdx.x; j < cols; j += 256) t += c[k * ldc + j];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc[k] += red[0];
}

// one thread per row r: g[r] += sum_j X(r, j) coef[j], columns in order
template <typename XT>
__global__ __launch_bounds__(256) void dosage_gemv_kernel(const XT* __restrict__ X, int64_t ldx, int64_t n,
                                                          int64_t cols, const double* __restrict__ coef,
                                                          double* __restrict__ g) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double t = 0.0;
    for (int64_t j = 0; j < cols; ++j) t += (double)X[j * ldx + r] * coef[j];
    g[r] += t;
}

}  // namespace

hipError_t snp_cross_w(int xt, const void* X, int64_t ldx, int64_t n, int64_t cols,
                       const double* W, int64_t ldw, int Qc, double* xw, int64_t ldxw,
                       hipStream_t s) {
    if (cols <= 0) return hipSuccess;
    if (!X || !W || !xw || ldx < n || ldw < n || ldxw < cols || Qc < 1) return hipErrorInvalidValue;
    const int64_t waves = (cols + XW_COLS - 1) / XW_COLS;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    if (xt == X_I8)
        hipLaunchKernelGGL(snp_cross_w_kernel<int8_t>, dim3(grid), dim3(256), 0, s,
                           (const int8_t*)X, ldx, n, cols, W, ldw, Qc, xw, ldxw);
    else
        hipLaunchKernelGGL(snp_cross_w_kernel<double>, dim3(grid), dim3(256), 0, s,
                           (const double*)X, ldx, n, cols, W, ldw, Qc, xw, ldxw);
    return hipGetLastError();
}

hipError_t snp_backward(const BackArgs& a, hipStream_t s) {
    if (a.cols <= 0) return hipSuccess;
    if (a.p < 2 || a.p > 20 || !a.part || !a.xw || !a.consts || !a.G || !a.gy0 || !a.b || !a.var ||
        !a.info || !a.gb || !a.contrib || !a.coef || a.ldc < a.cols || a.ldb < a.p || a.ldgb < a.p)
        return hipErrorInvalidValue;
    const unsigned grid = (unsigned)((a.cols + 127) / 128);
    switch (a.p - 1) {
#define GWAS_BACK_CASE(q) \
    case q: hipLaunchKernelGGL(snp_backward_kernel<q>, dim3(grid), dim3(128), 0, s, a); break;
        GWAS_BACK_CASE(1) GWAS_BACK_CASE(2) GWAS_BACK_CASE(3) GWAS_BACK_CASE(4)
        GWAS_BACK_CASE(5) GWAS_BACK_CASE(6) GWAS_BACK_CASE(7) GWAS_BACK_CASE(8)
        GWAS_BACK_CASE(9) GWAS_BACK_CASE(10) GWAS_BACK_CASE(11) GWAS_BACK_CASE(12)
        GWAS_BACK_CASE(13) GWAS_BACK_CASE(14) GWAS_BACK_CASE(15) GWAS_BACK_CASE(16)
        GWAS_BACK_CASE(17) GWAS_BACK_CASE(18) GWAS_BACK_CASE(19)
#undef GWAS_BACK_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t sum_columns(const double* contrib, int64_t ldc, int rows, int64_t cols, double* acc,
                       hipStream_t s) {
    if (cols <= 0 || rows <= 0) return hipSuccess;
    if (!contrib || !acc || ldc < cols) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sum_columns_kernel, dim3(rows), dim3(256), 0, s, contrib, ldc, cols, acc);
    return hipGetLastError();
}

hipError_t partial_chunks(const double* part, int64_t ldp, int64_t npb, int Q, int64_t cols, int chunk,
                          double* out, int64_t ldo, hipStream_t s) {
    if (cols <= 0) return hipSuccess;
    if (!part || !out || npb < 1 || Q < 1 || chunk < 1 || ldp < cols || ldo < cols) return hipErrorInvalidValue;
    const int64_t G = (npb + chunk - 1) / chunk;
    const int64_t threads = cols * Q * G;
    hipLaunchKernelGGL(partial_chunks_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, part, ldp,
                       npb, Q, cols, chunk, G, out, ldo);
    return hipGetLastError();
}

hipError_t dosage_gemv(int xt, const void* X, int64_t ldx, int64_t n, int64_t cols, const double* coef,
                       double* g, hipStream_t s) {
    if (cols <= 0) return hipSuccess;
    if (!X || !coef || !g || ldx < n) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)((n + 255) / 256);
    if (xt == X_I8)
        hipLaunchKernelGGL(dosage_gemv_kernel<int8_t>, dim3(grid), dim3(256), 0, s, (const int8_t*)X, ldx, n,
                           cols, coef, g);
    else
        hipLaunchKernelGGL(dosage_gemv_kernel<double>, dim3(grid), dim3(256), 0, s, (const double*)X, ldx, n,
                           cols, coef, g);
    return hipGetLastError();
}

hipError_t snp_solve(const SolveArgs& a, hipStream_t s) {
    if (a.cols <= 0) return hipSuccess;
    if (a.p < 2 || a.p > 20 || a.t < 1 || !a.part || !a.consts || !a.b || a.ldb < a.p * a.t)
        return hipErrorInvalidValue;
    if (!a.xw && a.Q != a.p + a.t) return hipErrorInvalidValue;
    if (a.xw && a.Q != 1) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)((a.cols + 127) / 128);
    switch (a.p - 1) {
#define GWAS_SOLVE_CASE(q) \
    case q: hipLaunchKernelGGL(snp_solve_kernel<q>, dim3(grid), dim3(128), 0, s, a); break;
        GWAS_SOLVE_CASE(1) GWAS_SOLVE_CASE(2) GWAS_SOLVE_CASE(3) GWAS_SOLVE_CASE(4)
        GWAS_SOLVE_CASE(5) GWAS_SOLVE_CASE(6) GWAS_SOLVE_CASE(7) GWAS_SOLVE_CASE(8)
        GWAS_SOLVE_CASE(9) GWAS_SOLVE_CASE(10) GWAS_SOLVE_CASE(11) GWAS_SOLVE_CASE(12)
        GWAS_SOLVE_CASE(13) GWAS_SOLVE_CASE(14) GWAS_SOLVE_CASE(15) GWAS_SOLVE_CASE(16)
        GWAS_SOLVE_CASE(17) GWAS_SOLVE_CASE(18) GWAS_SOLVE_CASE(19)
#undef GWAS_SOLVE_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gwas
