// Kernels run once per context: the float64 matrix-core product used by the
// recursive Cholesky / triangular inverse and the whitening of X_L and y
// (Algorithm 1, first three lines), the 64 x 64 diagonal-block factorisation
// in LDS, padding and conversion helpers, and the constant p x p blocks.
#include "internal.h"

#include <math.h>

#include <algorithm>

namespace gwas {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

constexpr int GBK = 16;        // K depth of one LDS stage
constexpr int GLD = GBK + 2;   // LDS row stride (doubles): 144 B keeps rows 16-B aligned

__device__ __forceinline__ d4_t mfma_f64(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 128 x GBK slab of an operand in registers: 8 doubles per thread.
// kcontig: element (r,k) at P[k + r*ld] (K contiguous); else P[r + k*ld].
__device__ __forceinline__ void load_slab(double (&v)[8], const double* __restrict__ P, int64_t ld,
                                          bool kcontig, int64_t r0, int64_t rlim, int64_t k0,
                                          int64_t klim, int tid) {
    if (kcontig) {
        const int r = tid >> 1, kk = (tid & 1) * 8;
        const int64_t row = r0 + r;
        if (row < rlim && k0 + kk + 8 <= klim) {
            const double* src = P + row * ld + k0 + kk;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = src[j];
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v[j] = (row < rlim && k0 + kk + j < klim) ? P[row * ld + k0 + kk + j] : 0.0;
        }
    } else {
        const int k = tid >> 4, rr = (tid & 15) * 8;
        const int64_t kk = k0 + k;
        if (kk < klim && r0 + rr + 8 <= rlim) {
            const double* src = P + kk * ld + r0 + rr;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = src[j];
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v[j] = (kk < klim && r0 + rr + j < rlim) ? P[kk * ld + r0 + rr + j] : 0.0;
        }
    }
}

__device__ __forceinline__ void store_slab(const double (&v)[8], double (*S)[GLD], bool kcontig,
                                           int tid) {
    if (kcontig) {
        const int r = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j) S[r][kk + j] = v[j];
    } else {
        const int k = tid >> 4, rr = (tid & 15) * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j) S[rr + j][k] = v[j];
    }
}

// One 128 x 128 tile per workgroup; four waves in a 2 x 2 grid, 64 x 64 each
// as 4 x 4 blocks of the 16x16x4 float64 matrix instruction.  Within a K
// stage, lane group g = lane/16 supplies k = 4g + s at instruction step s,
// for A and B alike, so every k of the stage is summed exactly once.
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmArgs g) {
    const int64_t m0 = (int64_t)blockIdx.x * TILE_M;
    const int64_t n0 = (int64_t)blockIdx.y * TILE_N;
    if (g.lower_only && m0 + TILE_M <= n0) return;

    int64_t kbeg = 0, kend = g.K;
    if (g.kflags & KR_A_LOWER) kend = min(kend, m0 + TILE_M);
    if (g.kflags & KR_B_UPPER) kend = min(kend, n0 + TILE_N);
    if (g.kflags & KR_A_UPPER) kbeg = max(kbeg, m0);
    if (g.kflags & KR_B_LOWER) kbeg = max(kbeg, n0);
    kbeg = (kbeg / GBK) * GBK;

    __shared__ double As[2][TILE_M][GLD];
    __shared__ double Bs[2][TILE_N][GLD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 15, lg = lane >> 4;
    const bool a_kc = (g.opA == 'T');
    const bool b_kc = (g.opB == 'N');

    d4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    const int64_t nk = (kend > kbeg) ? (kend - kbeg + GBK - 1) / GBK : 0;
    double ra[8], rb[8];
    if (nk > 0) {
        load_slab(ra, g.A, g.lda, a_kc, m0, g.M, kbeg, kend, tid);
        load_slab(rb, g.B, g.ldb, b_kc, n0, g.N, kbeg, kend, tid);
        store_slab(ra, As[0], a_kc, tid);
        store_slab(rb, Bs[0], b_kc, tid);
    }
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) {
            const int64_t k0 = kbeg + (kt + 1) * GBK;
            load_slab(ra, g.A, g.lda, a_kc, m0, g.M, k0, kend, tid);
            load_slab(rb, g.B, g.ldb, b_kc, n0, g.N, k0, kend, tid);
        }
        d2_t av[4][2], bv[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const d2_t* pa = reinterpret_cast<const d2_t*>(&As[buf][wr * 64 + i * 16 + li][4 * lg]);
            av[i][0] = pa[0];
            av[i][1] = pa[1];
            const d2_t* pb = reinterpret_cast<const d2_t*>(&Bs[buf][wc * 64 + i * 16 + li][4 * lg]);
            bv[i][0] = pb[0];
            bv[i][1] = pb[1];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = mfma_f64(av[i][s >> 1][s & 1], bv[j][s >> 1][s & 1], acc[i][j]);
        if (more) {
            store_slab(ra, As[buf ^ 1], a_kc, tid);
            store_slab(rb, Bs[buf ^ 1], b_kc, tid);
        }
        __syncthreads();
    }

    // D of the 16x16x4 float64 instruction: element v of a lane holds row
    // lane/16 + 4v, column lane%16.
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t col = n0 + wc * 64 + j * 16 + li;
            if (col >= g.N) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = m0 + wr * 64 + i * 16 + lg + 4 * v;
                if (row >= g.M) continue;
                double* c = g.C + row + col * g.ldc;
                const double r = g.alpha * acc[i][j][v];
                *c = (g.beta == 0.0) ? r : r + g.beta * *c;
            }
        }
}

// Right-looking Cholesky of one LEAF x LEAF block by a single wave (lane i
// owns row i), then its inverse by forward substitution (lane c owns column
// c of L^-1).  The block lives in LDS.
__global__ __launch_bounds__(64) void chol_leaf_kernel(double* L, double* U, int64_t ld,
                                                       int64_t row0, int64_t n_valid, int* fail) {
    __shared__ double A[LEAF][LEAF + 1];
    __shared__ double X[LEAF][LEAF + 1];
    const int i = threadIdx.x;
    for (int c = 0; c < LEAF; ++c) A[i][c] = (c <= i) ? L[i + c * ld] : 0.0;
    __syncthreads();
    for (int j = 0; j < LEAF; ++j) {
        const double d = A[j][j];
        const bool bad = !(d > 0.0);
        if (bad && i == j && row0 + j < n_valid) atomicMin(fail, (int)(row0 + j + 1));
        const double piv = sqrt(d);   // NaN on failure, which propagates
        __syncthreads();
        if (i > j) A[i][j] /= piv;
        if (i == j) A[j][j] = piv;
        __syncthreads();
        if (i > j) {
            const double lij = A[i][j];
            for (int k = j + 1; k <= i; ++k) A[i][k] -= lij * A[k][j];
        }
        __syncthreads();
    }
    // column c of L^-1: x_r = (delta_rc - sum_{k=c}^{r-1} L(r,k) x_k) / L(r,r)
    {
        const int c = i;
        for (int r = 0; r < LEAF; ++r) {
            double x = 0.0;
            if (r >= c) {
                double s = (r == c) ? 1.0 : 0.0;
                for (int k = c; k < r; ++k) s -= A[r][k] * X[k][c];
                x = s / A[r][r];
            }
            X[r][c] = x;
        }
    }
    __syncthreads();
    // write L (zero above the diagonal) and U = L^-T (zero below)
    for (int c = 0; c < LEAF; ++c) {
        L[i + c * ld] = (c <= i) ? A[i][c] : 0.0;
        U[i + c * ld] = X[c][i];     // U(i,c) = L^-1(c,i), zero for i > c
    }
}

// one workgroup per column (grid-stride over columns), threads over rows
__global__ void pad_identity_kernel(double* A, int64_t ld, int64_t n, int64_t n_pad) {
    for (int64_t c = blockIdx.x; c < n_pad; c += gridDim.x) {
        const int64_t r0 = (c < n) ? n : 0;
        for (int64_t r = r0 + threadIdx.x; r < n_pad; r += blockDim.x)
            A[r + c * ld] = (r == c) ? 1.0 : 0.0;
    }
}

template <typename T>
__global__ void convert_kernel(const double* __restrict__ in, T* __restrict__ out, int64_t ld,
                               int64_t rows, int64_t cols) {
    for (int64_t c = blockIdx.x; c < cols; c += gridDim.x)
        for (int64_t r = threadIdx.x; r < rows; r += blockDim.x)
            out[r + c * ld] = (T)in[r + c * ld];
}

// One workgroup per row of L^-1 (grid-stride): block max, power-of-two
// scale, then exact 7-bit digits (every step is a multiplication by a power
// of two or the subtraction of a nearby integer, so no rounding occurs).
__global__ __launch_bounds__(256) void slice_rows_kernel(const double* __restrict__ U, int64_t ld,
                                                         int64_t n_pad, int S, int8_t* __restrict__ A,
                                                         int64_t lda, double* __restrict__ rscale) {
    __shared__ double red[256];
    for (int64_t r = blockIdx.x; r < n_pad; r += gridDim.x) {
        const double* col = U + r * ld;      // L^-1(r, k) = U(k, r), zero for k > r
        double m = 0.0;
        for (int64_t k = threadIdx.x; k <= r; k += blockDim.x) m = fmax(m, fabs(col[k]));
        red[threadIdx.x] = m;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        m = red[0];
        __syncthreads();
        int e = 0;
        if (m > 0.0) (void)frexp(m, &e);        // m < 2^e
        const double sc = ldexp(1.0, e);
        if (threadIdx.x == 0) rscale[r] = sc;
        const int64_t base = (r / 16) * 16 * S + (r % 16);
        for (int64_t k = threadIdx.x; k < n_pad; k += blockDim.x) {
            double t = (k <= r) ? ldexp(col[k], 6 - e) : 0.0;   // (L^-1(r,k)/sc) * 2^6, |t| <= 64
            for (int sl = 0; sl < S; ++sl) {
                const double q = rint(t);
                A[(base + sl * 16) * lda + k] = (int8_t)q;
                t = (t - q) * 128.0;
            }
        }
    }
}

// R = chol(S_TL), v = R^-1 bbar_T; single thread (q1 <= 19).
__global__ void snp_constants_kernel(const double* S, int64_t lds, int q1, int t, double* K,
                                     int* fail) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double* R = K + consts_R(q1);
    double* v = K + consts_v(q1);
    double* STL = K + consts_STL(q1, t);
    double* bT = K + consts_bT(q1, t);
    for (int c = 0; c < q1; ++c)
        for (int r = 0; r < q1; ++r) {
            STL[r + c * q1] = S[r + c * lds];
            R[r + c * q1] = (r >= c) ? S[r + c * lds] : 0.0;
        }
    for (int j = 0; j < t; ++j)
        for (int r = 0; r < q1; ++r) bT[r + j * q1] = S[r + (q1 + j) * lds];
    int f = 0;
    for (int j = 0; j < q1; ++j) {
        double d = R[j + j * q1];
        for (int k = 0; k < j; ++k) d -= R[j + k * q1] * R[j + k * q1];
        // a pivot that keeps no more than 1e-10 of its diagonal entry means
        // X_L is numerically rank deficient
        if (!(d > 1e-10 * STL[j + j * q1]) && f == 0) f = j + 1;
        d = sqrt(d);
        R[j + j * q1] = d;
        for (int r = j + 1; r < q1; ++r) {
            double s = R[r + j * q1];
            for (int k = 0; k < j; ++k) s -= R[r + k * q1] * R[j + k * q1];
            R[r + j * q1] = s / d;
        }
    }
    for (int j = 0; j < t; ++j)
        for (int r = 0; r < q1; ++r) {
            double s = bT[r + j * q1];
            for (int k = 0; k < r; ++k) s -= R[r + k * q1] * v[k + j * q1];
            v[r + j * q1] = s / R[r + r * q1];
        }
    *fail = f;
}

}  // namespace

hipError_t gemm_f64(const GemmArgs& g, hipStream_t s) {
    if (g.M < 0 || g.N < 0 || g.K < 0) return hipErrorInvalidValue;
    if (g.M == 0 || g.N == 0) return hipSuccess;
    if (!g.A || !g.B || !g.C) return hipErrorInvalidValue;
    if ((g.opA != 'N' && g.opA != 'T') || (g.opB != 'N' && g.opB != 'T')) return hipErrorInvalidValue;
    if (g.ldc < g.M) return hipErrorInvalidValue;
    if (g.opA == 'N' ? g.lda < g.M : g.lda < g.K) return hipErrorInvalidValue;
    if (g.opB == 'N' ? g.ldb < g.K : g.ldb < g.N) return hipErrorInvalidValue;
    dim3 grid((unsigned)((g.M + TILE_M - 1) / TILE_M), (unsigned)((g.N + TILE_N - 1) / TILE_N));
    if (grid.y > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t chol_leaf(double* L, double* U, int64_t ld, int64_t row0, int64_t n_valid, int* fail,
                     hipStream_t s) {
    if (!L || !U || !fail || ld < LEAF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chol_leaf_kernel, dim3(1), dim3(LEAF), 0, s, L, U, ld, row0, n_valid, fail);
    return hipGetLastError();
}

hipError_t pad_identity(double* A, int64_t ld, int64_t n, int64_t n_pad, hipStream_t s) {
    if (n_pad <= 0 || n < 0 || n > n_pad || ld < n_pad) return hipErrorInvalidValue;
    if (n == n_pad) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>(n_pad, 8192);
    hipLaunchKernelGGL(pad_identity_kernel, dim3(grid), dim3(256), 0, s, A, ld, n, n_pad);
    return hipGetLastError();
}

hipError_t convert_f32(const double* in, float* out, int64_t ld, int64_t rows, int64_t cols,
                       hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (ld < rows) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<int64_t>(cols, 8192);
    hipLaunchKernelGGL(convert_kernel<float>, dim3(grid), dim3(256), 0, s, in, out, ld, rows, cols);
    return hipGetLastError();
}

hipError_t convert_bf16(const double* in, __bf16* out, int64_t ld, int64_t rows, int64_t cols,
                        hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (ld < rows) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<int64_t>(cols, 8192);
    hipLaunchKernelGGL(convert_kernel<__bf16>, dim3(grid), dim3(256), 0, s, in, out, ld, rows, cols);
    return hipGetLastError();
}

hipError_t slice_rows(const double* U, int64_t ld, int64_t n_pad, int S, int8_t* A, int64_t lda,
                      double* rscale, hipStream_t s) {
    if (!U || !A || !rscale || S < 1 || S > 8 || ld < n_pad || lda < n_pad || n_pad % 16)
        return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<int64_t>(n_pad, 16384);
    hipLaunchKernelGGL(slice_rows_kernel, dim3(grid), dim3(256), 0, s, U, ld, n_pad, S, A, lda, rscale);
    return hipGetLastError();
}

hipError_t snp_constants(const double* S, int64_t lds, int q1, int t, double* consts, int* fail,
                         hipStream_t s) {
    if (q1 < 1 || q1 > 19 || t < 1 || lds < q1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(snp_constants_kernel, dim3(1), dim3(64), 0, s, S, lds, q1, t, consts, fail);
    return hipGetLastError();
}

}  // namespace gwas
