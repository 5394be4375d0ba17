// Per-SNP kernels of the per-block hot path (Algorithm 2, loop body) and of
// its reverse pass:
//   snp_cross_w     x^T W with W = M^-1 [X_L | y] on the float64 matrix cores
//                   (reduced-precision paths and the reverse pass);
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

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u2_t __attribute__((ext_vector_type(2)));

// x_j^T W[:, q] on the float64 matrix cores: C (SNPs x Qc) = X^T W with K = n.
// A workgroup of WV waves (4, or 1 for narrow blocks, which then get four
// times the workgroups) takes 64 WV SNPs (a wave 64, as 4 blocks of 16) and
// WQ blocks of 16 columns of W, over one K split of klen rows (XW_KSPLIT,
// or all of n in a single split).  The splits depend on n alone, so the sums
// of a SNP do not depend on the block it comes in; with several splits each
// writes its partial sums and xw_reduce_kernel adds them in split order.  Stages of 16 k go through
// LDS: a thread's dosage chunk is one SNP's 16 k, loaded whole when its
// first element is below n (inside the array, since ldx bytes are a
// multiple of 16) and cleared past n in registers.
constexpr int XW_BK = 16;
constexpr int XW_KSPLIT = 2048;
constexpr int XW_QMAX = 80;         // columns of W per workgroup (5 blocks)

template <typename XT, int WQ, int WV>
__global__ __launch_bounds__(64 * WV) void xw_kernel(const XT* X, int64_t ldx, int64_t n,
                                                           int64_t cols, const double* __restrict__ W,
                                                           int64_t ldw, int Qc, double* __restrict__ out,
                                                           int64_t ldo, int64_t split_stride, int64_t klen,
                                                           int check012, const TrmmArgs* xargs) {
    // xargs: the dosages' address and stride come from a device argument
    // array (a replayed graph reads the block's dosages in place)
    if (xargs) {
        X = static_cast<const XT*>(xargs->Xd);
        ldx = xargs->ldxd;
    }
    constexpr int NT = 64 * WV;
    constexpr int TC = 64 * WV;                     // SNPs per workgroup, one per thread
    constexpr int TQ = 16 * WQ;
    constexpr int XLD = sizeof(XT) == 1 ? XW_BK : XW_BK + 1;   // LDS row of a SNP (elements)
    constexpr int WLD = XW_BK + 1;                  // LDS row of a column of W (doubles)
    constexpr int CPC = XW_BK * (int)sizeof(XT) / 16;          // 16-byte chunks per SNP per stage
    constexpr int EPC = 16 / (int)sizeof(XT);
    __shared__ __attribute__((aligned(16))) XT Xs[2][TC * XLD];
    __shared__ double Ws[2][TQ * WLD];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t c0 = (int64_t)blockIdx.x * TC;
    const int split = blockIdx.y;
    const int q0 = blockIdx.z * TQ;
    const int64_t kbeg = (int64_t)split * klen;
    const int64_t kend = std::min<int64_t>(n, kbeg + klen);
    const int nst = (int)((kend - kbeg + XW_BK - 1) / XW_BK);

    u4_t rx[CPC];
    double rw[(TQ * XW_BK / 2 + NT - 1) / NT][2];
    // check012: int8 dosages outside {0, 1, 2} in this thread's SNP (bytes
    // with a bit above bit 1 set, or both low bits)
    uint32_t bad = 0;
    auto load = [&](int st) {
        const int64_t k0 = kbeg + (int64_t)st * XW_BK;
        const int64_t col = c0 + tid;
#pragma unroll
        for (int c = 0; c < CPC; ++c) {
            const int64_t kc = k0 + c * EPC;
            u4_t v = u4_t{0u, 0u, 0u, 0u};
            if (col < cols && kc < n) v = *reinterpret_cast<const u4_t*>(X + col * ldx + kc);
            if (kc + EPC > n) {
                const int vb = (int)std::min<int64_t>(16, std::max<int64_t>(0, (n - kc) * (int64_t)sizeof(XT)));
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int keep = std::min(4, std::max(0, vb - 4 * w));
                    v[w] &= keep >= 4 ? 0xffffffffu : ((1u << (8 * keep)) - 1u);
                }
            }
            rx[c] = v;
            if constexpr (sizeof(XT) == 1) {
                if (check012) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) bad |= (v[w] & 0xfcfcfcfcu) | (v[w] & (v[w] >> 1) & 0x01010101u);
                }
            }
        }
        // W rows k0..k0+15 lie below n_pad = ldw, zero past n
#pragma unroll
        for (int c = 0; c < (TQ * XW_BK / 2 + NT - 1) / NT; ++c) {
            const int idx = tid + c * NT;
            const int q = idx / (XW_BK / 2), kk = (idx % (XW_BK / 2)) * 2;
            const bool ok = idx < TQ * XW_BK / 2 && q0 + q < Qc;
            const double* src = W + (q0 + q) * ldw + k0 + kk;
            rw[c][0] = ok ? src[0] : 0.0;
            rw[c][1] = ok ? src[1] : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < CPC; ++c) {
            if constexpr (sizeof(XT) == 1) {
                *reinterpret_cast<u4_t*>(Xs[buf] + tid * XLD + c * EPC) = rx[c];
            } else {
                // the chunk's two doubles, by value (elements copied to
                // scalars before the bit cast)
                const uint32_t w0 = rx[c][0], w1 = rx[c][1], w2 = rx[c][2], w3 = rx[c][3];
                Xs[buf][tid * XLD + c * EPC] = __builtin_bit_cast(double, u2_t{w0, w1});
                Xs[buf][tid * XLD + c * EPC + 1] = __builtin_bit_cast(double, u2_t{w2, w3});
            }
        }
#pragma unroll
        for (int c = 0; c < (TQ * XW_BK / 2 + NT - 1) / NT; ++c) {
            const int idx = tid + c * NT;
            if (idx < TQ * XW_BK / 2) {
                const int q = idx / (XW_BK / 2), kk = (idx % (XW_BK / 2)) * 2;
                Ws[buf][q * WLD + kk] = rw[c][0];
                Ws[buf][q * WLD + kk + 1] = rw[c][1];
            }
        }
    };

    d4_t acc[4][WQ];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int qb = 0; qb < WQ; ++qb) acc[cb][qb] = d4_t{0.0, 0.0, 0.0, 0.0};

    load(0);
    store(0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        const bool more = st + 1 < nst;
        if (more) load(st + 1);
        // lane group g supplies k = 4 step + g of the stage to both operands
#pragma unroll
        for (int step = 0; step < XW_BK / 4; ++step) {
            const int k = 4 * step + lg;
            double a[4], b[WQ];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) a[cb] = (double)Xs[buf][(wave * 64 + cb * 16 + li) * XLD + k];
#pragma unroll
            for (int qb = 0; qb < WQ; ++qb) b[qb] = Ws[buf][(qb * 16 + li) * WLD + k];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int qb = 0; qb < WQ; ++qb)
                    acc[cb][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cb], b[qb], acc[cb][qb], 0, 0, 0);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
    }
    // a SNP with a dosage outside {0, 1, 2} gets NaN cross products (the
    // centred int8 product cannot represent it)
    __shared__ int badS[TC];
    if (check012) {
        badS[tid] = bad != 0;
        __syncthreads();
    }
    // element v of a lane: SNP (A row) lane/16 + 4v of the block, column of
    // W (B column) lane%16
    double* o = out + (int64_t)split * split_stride;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int qb = 0; qb < WQ; ++qb) {
            const int q = q0 + qb * 16 + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int lc = wave * 64 + cb * 16 + lg + 4 * v;
                const int64_t col = c0 + lc;
                const double val = (check012 && badS[lc]) ? __builtin_nan("") : acc[cb][qb][v];
                if (q < Qc && col < cols) o[(int64_t)q * ldo + col] = val;
            }
        }
}

// xw[q * ldxw + j] = sum over splits, in split order, of the partial sums.
__global__ __launch_bounds__(256) void xw_reduce_kernel(const double* __restrict__ part, int splits, int Qc,
                                                        int64_t cols, double* __restrict__ xw, int64_t ldxw) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)Qc * cols) return;
    const int64_t q = i / cols, j = i % cols;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += part[((int64_t)sp * Qc + q) * cols + j];
    xw[q * ldxw + j] = s;
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

int xw_splits(int64_t n) { return (int)std::max<int64_t>(1, (n + XW_KSPLIT - 1) / XW_KSPLIT); }

hipError_t snp_cross_w(int xt, const void* X, int64_t ldx, int64_t n, int64_t cols,
                       const double* W, int64_t ldw, int Qc, double* xw, int64_t ldxw,
                       double* part, int64_t part_cap, hipStream_t s, bool check012,
                       const TrmmArgs* xargs) {
    if (cols <= 0) return hipSuccess;
    if (!X || !W || !xw || n < 1 || ldx < n || ldw < (n + XW_BK - 1) / XW_BK * XW_BK || ldxw < cols || Qc < 1)
        return hipErrorInvalidValue;
    const size_t xs = xt == X_I8 ? 1 : 8;
    if ((reinterpret_cast<uintptr_t>(X) % 16) || ((ldx * (int64_t)xs) % 16)) return hipErrorInvalidValue;
    // K splits: from n alone when there is room for the partial sums
    const int splits = part ? xw_splits(n) : 1;
    if (splits > 1 && part_cap < (int64_t)splits * Qc * cols) return hipErrorInvalidValue;
    const int qchunks = (Qc + XW_QMAX - 1) / XW_QMAX;
    const int wq = qchunks > 1 ? XW_QMAX / 16 : (Qc + 15) / 16;
    // one-wave workgroups when four-wave ones would not fill the chip; every
    // sum runs over the same K steps either way
    const bool narrow = (cols + 255) / 256 * splits * qchunks < 1024;
    const int wv = narrow ? 1 : 4;
    const dim3 grid((unsigned)((cols + 64 * wv - 1) / (64 * wv)), (unsigned)splits, (unsigned)qchunks);
    double* out = splits > 1 ? part : xw;
    const int64_t ldo = splits > 1 ? cols : ldxw;
    const int64_t stride = splits > 1 ? (int64_t)Qc * cols : 0;
    // rows of X per split: a multiple of XW_BK, so only the last split is ragged
    const int64_t klen = splits > 1 ? (int64_t)XW_KSPLIT : (n + XW_BK - 1) / XW_BK * XW_BK;
#define GWAS_XW(T, WQ)                                                                                 \
    if (narrow) hipLaunchKernelGGL((xw_kernel<T, WQ, 1>), grid, dim3(64), 0, s, (const T*)X, ldx, n, cols, \
                                   W, ldw, Qc, out, ldo, stride, klen, (int)(check012 && xt == X_I8), xargs); \
    else hipLaunchKernelGGL((xw_kernel<T, WQ, 4>), grid, dim3(256), 0, s, (const T*)X, ldx, n, cols, \
                       W, ldw, Qc, out, ldo, stride, klen, (int)(check012 && xt == X_I8), xargs)
#define GWAS_XW_T(T)                        \
    switch (wq) {                           \
        case 1: GWAS_XW(T, 1); break;       \
        case 2: GWAS_XW(T, 2); break;       \
        case 3: GWAS_XW(T, 3); break;       \
        case 4: GWAS_XW(T, 4); break;       \
        default: GWAS_XW(T, 5); break;      \
    }
    if (xt == X_I8) {
        GWAS_XW_T(int8_t)
    } else {
        GWAS_XW_T(double)
    }
#undef GWAS_XW_T
#undef GWAS_XW
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    const int64_t total = (int64_t)Qc * cols;
    hipLaunchKernelGGL(xw_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, part, splits, Qc,
                       cols, xw, ldxw);
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
