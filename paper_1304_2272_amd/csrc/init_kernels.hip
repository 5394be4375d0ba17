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

// R x GBK slab of an operand, moved global -> registers -> LDS in 16-byte
// chunks of two doubles.  kcontig: element (r,k) at P[k + r*ld]; otherwise at
// P[r + k*ld] (and the chunk is two consecutive r, stored transposed).
// Out-of-range elements are zero; `vec` allows 16-byte loads (ld even and P
// 16-byte aligned).
template <int R, int NT> struct Slab {
    static constexpr int CH = R * GBK / 2;           // chunks per stage
    static constexpr int PER = (CH + NT - 1) / NT;
    d2_t v[PER];
};

template <int R, int NT, bool kcontig>
__device__ __forceinline__ void load_slab(Slab<R, NT>& sl, const double* __restrict__ P, int64_t ld,
                                          bool vec, int64_t r0, int64_t rlim, int64_t k0,
                                          int64_t klim, int tid) {
    // Whole slab inside the operand: one branch for the workgroup and plain
    // 16-byte loads (the per-chunk checks below keep the compiler from
    // overlapping the loads).
    if (vec && r0 + R <= rlim && k0 + GBK <= klim) {
#pragma unroll
        for (int c = 0; c < Slab<R, NT>::PER; ++c) {
            const int idx = tid + c * NT;
            if (Slab<R, NT>::CH % NT != 0 && idx >= Slab<R, NT>::CH) break;
            if constexpr (kcontig)
                sl.v[c] = *reinterpret_cast<const d2_t*>(P + (r0 + idx / (GBK / 2)) * ld + k0 + (idx % (GBK / 2)) * 2);
            else
                sl.v[c] = *reinterpret_cast<const d2_t*>(P + (k0 + idx / (R / 2)) * ld + r0 + (idx % (R / 2)) * 2);
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < Slab<R, NT>::PER; ++c) {
        const int idx = tid + c * NT;
        if (Slab<R, NT>::CH % NT != 0 && idx >= Slab<R, NT>::CH) break;
        int64_t r, k;
        if constexpr (kcontig) {
            r = r0 + idx / (GBK / 2);
            k = k0 + (idx % (GBK / 2)) * 2;
            if (vec && r < rlim && k + 2 <= klim) {
                sl.v[c] = *reinterpret_cast<const d2_t*>(P + r * ld + k);
            } else {
                sl.v[c][0] = (r < rlim && k < klim) ? P[r * ld + k] : 0.0;
                sl.v[c][1] = (r < rlim && k + 1 < klim) ? P[r * ld + k + 1] : 0.0;
            }
        } else {
            k = k0 + idx / (R / 2);
            r = r0 + (idx % (R / 2)) * 2;
            if (vec && k < klim && r + 2 <= rlim) {
                sl.v[c] = *reinterpret_cast<const d2_t*>(P + k * ld + r);
            } else {
                sl.v[c][0] = (k < klim && r < rlim) ? P[k * ld + r] : 0.0;
                sl.v[c][1] = (k < klim && r + 1 < rlim) ? P[k * ld + r + 1] : 0.0;
            }
        }
    }
}

// LDS image of one operand's stage.  kcontig operands keep rows of K
// (R x GLD); the others keep their global layout, rows of R at fixed k
// (GBK x (R + 2)), so both are written in 16-byte chunks and a lane's
// fragment is one 16-byte read (kcontig) or two 8-byte reads of
// consecutive k, 16 lanes over consecutive r (the others).
template <int R, bool kcontig> struct Lds {
    static constexpr int SIZE = kcontig ? R * GLD : GBK * (R + 2);
    __device__ static d2_t frag(const double* S, int r, int k) {
        if constexpr (kcontig) {
            return *reinterpret_cast<const d2_t*>(S + r * GLD + k);
        } else {
            return d2_t{S[k * (R + 2) + r], S[(k + 1) * (R + 2) + r]};
        }
    }
};

template <int R, int NT, bool kcontig>
__device__ __forceinline__ void store_slab(const Slab<R, NT>& sl, double* S, int tid) {
#pragma unroll
    for (int c = 0; c < Slab<R, NT>::PER; ++c) {
        const int idx = tid + c * NT;
        if (Slab<R, NT>::CH % NT != 0 && idx >= Slab<R, NT>::CH) break;
        if constexpr (kcontig) {
            *reinterpret_cast<d2_t*>(S + (idx / (GBK / 2)) * GLD + (idx % (GBK / 2)) * 2) = sl.v[c];
        } else {
            const int k = idx / (R / 2), r = (idx % (R / 2)) * 2;
            *reinterpret_cast<d2_t*>(S + k * (R + 2) + r) = sl.v[c];
        }
    }
}

// One 128 x (WGN*64) tile per workgroup of 2 x WGN waves, 64 x 64 each as
// 4 x 4 blocks of the 16x16x4 float64 matrix instruction.  Within a K stage,
// lane group g = lane/16 supplies k = 4g + s at instruction step s, for A
// and B alike, so every k of the stage is summed exactly once.
template <int WGN, bool A_KC, bool B_KC>
__global__ __launch_bounds__(128 * WGN, (WGN == 2 ? 2 : 1)) void gemm_f64_kernel(GemmArgs g, int avec,
                                                                                 int bvec) {
    constexpr int NT = 128 * WGN;
    constexpr int TN = 64 * WGN;
    const int64_t m0 = (int64_t)blockIdx.x * TILE_M;
    const int64_t n0 = (int64_t)blockIdx.y * TN;
    if (g.lower_only && m0 + TILE_M <= n0) return;

    int64_t kbeg = 0, kend = g.K;
    if (g.kflags & KR_A_LOWER) kend = min(kend, m0 + TILE_M);
    if (g.kflags & KR_B_UPPER) kend = min(kend, n0 + TN);
    if (g.kflags & KR_A_UPPER) kbeg = max(kbeg, m0);
    if (g.kflags & KR_B_LOWER) kbeg = max(kbeg, n0);
    kbeg = (kbeg / GBK) * GBK;

    typedef Lds<TILE_M, A_KC> LA;
    typedef Lds<TN, B_KC> LB;
    __shared__ __attribute__((aligned(16))) double As[2][LA::SIZE];
    __shared__ __attribute__((aligned(16))) double Bs[2][LB::SIZE];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WGN, wc = wave % WGN;
    const int li = lane & 15, lg = lane >> 4;

    d4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    const int64_t nk = (kend > kbeg) ? (kend - kbeg + GBK - 1) / GBK : 0;
    Slab<TILE_M, NT> ra;
    Slab<TN, NT> rb;
    if (nk > 0) {
        load_slab<TILE_M, NT, A_KC>(ra, g.A, g.lda, avec, m0, g.M, kbeg, kend, tid);
        load_slab<TN, NT, B_KC>(rb, g.B, g.ldb, bvec, n0, g.N, kbeg, kend, tid);
        store_slab<TILE_M, NT, A_KC>(ra, As[0], tid);
        store_slab<TN, NT, B_KC>(rb, Bs[0], tid);
    }
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        const bool more = kt + 1 < nk;
        // vmcnt(0), already met: the previous stage's loads went to LDS before
        // its barrier.  Without it the compiler assumes loads of other paths
        // may be in flight and waits between this stage's loads.
        __builtin_amdgcn_s_waitcnt(0x0f70);
        if (more) {
            const int64_t k0 = kbeg + (kt + 1) * GBK;
            load_slab<TILE_M, NT, A_KC>(ra, g.A, g.lda, avec, m0, g.M, k0, kend, tid);
            load_slab<TN, NT, B_KC>(rb, g.B, g.ldb, bvec, n0, g.N, k0, kend, tid);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            d2_t av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                av[i] = LA::frag(As[buf], wr * 64 + i * 16 + li, 4 * lg + 2 * h);
                bv[i] = LB::frag(Bs[buf], wc * 64 + i * 16 + li, 4 * lg + 2 * h);
            }
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = mfma_f64(av[i][s], bv[j][s], acc[i][j]);
        }
        if (more) {
            store_slab<TILE_M, NT, A_KC>(ra, As[buf ^ 1], tid);
            store_slab<TN, NT, B_KC>(rb, Bs[buf ^ 1], tid);
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
    // The whole LEAF x LEAF block lies inside the matrix: its loads are issued
    // together and waited for once (a load per element behind its own branch
    // waited for each in turn), then the lower triangle is kept.
    double v[LEAF];
#pragma unroll
    for (int c = 0; c < LEAF; ++c) v[c] = L[i + c * ld];
#pragma unroll
    for (int c = 0; c < LEAF; ++c) A[i][c] = (c <= i) ? v[c] : 0.0;
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
            // iterations are independent: unrolled, their LDS reads overlap
#pragma unroll 8
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
#pragma unroll 8
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

// Three bfloat16 slices of each row of L^-1: slice i is what slices 0..i-1
// leave of U(k, r), rounded to bfloat16 (every remainder is exact in
// float64), written to out[k + i*n_pad + r*ldo].
__global__ void slice_bf16_kernel(const double* __restrict__ U, int64_t ld, int64_t n_pad,
                                  __bf16* __restrict__ out, int64_t ldo) {
    for (int64_t r = blockIdx.x; r < n_pad; r += gridDim.x)
        for (int64_t k = threadIdx.x; k < n_pad; k += blockDim.x) {
            double v = U[k + r * ld];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const __bf16 h = (__bf16)v;
                out[k + i * n_pad + r * ldo] = h;
                v -= (double)h;
            }
        }
}

// Float64 dosage columns cut the same way, zero from row n on.
__global__ void slice_x_bf16_kernel(const double* __restrict__ X, int64_t ldx, int64_t n, int64_t n_pad,
                                    int64_t cols, __bf16* __restrict__ out, int64_t ldo, const TrmmArgs* xargs) {
    if (xargs) {
        X = static_cast<const double*>(xargs->Xd);
        ldx = xargs->ldxd;
    }
    for (int64_t j = blockIdx.x; j < cols; j += gridDim.x)
        for (int64_t k = threadIdx.x; k < n_pad; k += blockDim.x) {
            double v = k < n ? X[k + j * ldx] : 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const __bf16 h = (__bf16)v;
                out[k + i * n_pad + j * ldo] = h;
                v -= (double)h;
            }
        }
}

__global__ void convert_x_bf16_kernel(const double* __restrict__ X, int64_t ldx, int64_t n, int64_t n_pad,
                                      int64_t cols, __bf16* __restrict__ out, int64_t ldo, const TrmmArgs* xargs) {
    if (xargs) {
        X = static_cast<const double*>(xargs->Xd);
        ldx = xargs->ldxd;
    }
    for (int64_t j = blockIdx.x; j < cols; j += gridDim.x)
        for (int64_t k = threadIdx.x; k < n_pad; k += blockDim.x)
            out[k + j * ldo] = k < n ? (__bf16)(float)X[k + j * ldx] : (__bf16)0.f;
}

// One workgroup per row of L^-1 (grid-stride): block max, power-of-two
// scale, then int8 digits in pairs: each digit rounds what the ones before
// it leave, scaled by 127 inside a pair and by 128 from one pair to the
// next (a subtraction of a nearby integer is exact; the scaling by 127
// rounds at 2^-53 of the digit, far below the last digit's half unit).
// The row sums 127 sum_{k<n} A_hi of the hi digits of each pair are exact
// int32 sums (|127 A_hi| <= 8,128, n < 2^18).
__global__ __launch_bounds__(256) void slice_rows_kernel(const double* __restrict__ U, int64_t ld,
                                                         int64_t n_pad, int64_t n, int S,
                                                         int8_t* __restrict__ A, int64_t lda,
                                                         double* __restrict__ rscale, int* __restrict__ rsum) {
    __shared__ double red[256];
    __shared__ int ired[SLICE_PAIRS_MAX][256];
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
        int dsum[SLICE_PAIRS_MAX] = {0, 0, 0};
        for (int64_t k = threadIdx.x; k < n_pad; k += blockDim.x) {
            double t = (k <= r) ? ldexp(col[k], 6 - e) : 0.0;   // (L^-1(r,k)/sc) * 2^6, |t| < 64
            for (int sl = 0; sl < S; ++sl) {
                const double q = rint(t);
                A[(base + sl * 16) * lda + k] = (int8_t)q;
                if (k < n && !(sl & 1) && sl / 2 < SLICE_PAIRS_MAX) dsum[sl / 2] += 127 * (int)q;
                t = (t - q) * ((sl & 1) ? 128.0 : 127.0);
            }
        }
        for (int p = 0; p < SLICE_PAIRS_MAX; ++p) ired[p][threadIdx.x] = dsum[p];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                for (int p = 0; p < SLICE_PAIRS_MAX; ++p) ired[p][threadIdx.x] += ired[p][threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x < (S + 1) / 2) rsum[threadIdx.x * n_pad + r] = ired[threadIdx.x][0];
        __syncthreads();
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
    const int avec = (g.lda % 2 == 0) && (reinterpret_cast<uintptr_t>(g.A) % 16 == 0);
    const int bvec = (g.ldb % 2 == 0) && (reinterpret_cast<uintptr_t>(g.B) % 16 == 0);
    const bool akc = g.opA == 'T', bkc = g.opB == 'N';
    const bool wide = g.N >= 256;
    dim3 grid((unsigned)((g.M + TILE_M - 1) / TILE_M), (unsigned)((g.N + (wide ? 255 : 127)) / (wide ? 256 : 128)));
    if (grid.y > 65535) return hipErrorInvalidValue;
#define GWAS_GEMM_LAUNCH(W, AK, BK)                                                              \
    hipLaunchKernelGGL((gemm_f64_kernel<W, AK, BK>), grid, dim3(128 * W), 0, s, g, avec, bvec)
    if (wide) {
        if (akc && bkc) GWAS_GEMM_LAUNCH(4, true, true);
        else if (akc) GWAS_GEMM_LAUNCH(4, true, false);
        else if (bkc) GWAS_GEMM_LAUNCH(4, false, true);
        else GWAS_GEMM_LAUNCH(4, false, false);
    } else {
        if (akc && bkc) GWAS_GEMM_LAUNCH(2, true, true);
        else if (akc) GWAS_GEMM_LAUNCH(2, true, false);
        else if (bkc) GWAS_GEMM_LAUNCH(2, false, true);
        else GWAS_GEMM_LAUNCH(2, false, false);
    }
#undef GWAS_GEMM_LAUNCH
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

hipError_t slice_bf16(const double* U, int64_t ld, int64_t n_pad, __bf16* out, int64_t ldo, hipStream_t s) {
    if (!U || !out || ld < n_pad || ldo < 3 * n_pad) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<int64_t>(n_pad, 8192);
    hipLaunchKernelGGL(slice_bf16_kernel, dim3(grid), dim3(256), 0, s, U, ld, n_pad, out, ldo);
    return hipGetLastError();
}

hipError_t slice_x_bf16(const double* X, int64_t ldx, int64_t n, int64_t n_pad, int64_t cols, __bf16* out,
                        int64_t ldo, hipStream_t s, const TrmmArgs* xargs) {
    if (cols <= 0) return hipSuccess;
    if ((!X && !xargs) || !out || n < 1 || n > n_pad || (!xargs && ldx < n) || ldo < 3 * n_pad)
        return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<int64_t>(cols, 16384);
    hipLaunchKernelGGL(slice_x_bf16_kernel, dim3(grid), dim3(256), 0, s, X, ldx, n, n_pad, cols, out, ldo, xargs);
    return hipGetLastError();
}

hipError_t convert_x_bf16(const double* X, int64_t ldx, int64_t n, int64_t n_pad, int64_t cols, __bf16* out,
                          int64_t ldo, hipStream_t s, const TrmmArgs* xargs) {
    if (cols <= 0) return hipSuccess;
    if ((!X && !xargs) || !out || n < 1 || n > n_pad || (!xargs && ldx < n) || ldo < n_pad)
        return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<int64_t>(cols, 16384);
    hipLaunchKernelGGL(convert_x_bf16_kernel, dim3(grid), dim3(256), 0, s, X, ldx, n, n_pad, cols, out, ldo, xargs);
    return hipGetLastError();
}

hipError_t slice_rows(const double* U, int64_t ld, int64_t n_pad, int64_t n, int S, int8_t* A, int64_t lda,
                      double* rscale, int* rsum, hipStream_t s) {
    if (!U || !A || !rscale || !rsum || S < 1 || S > 2 * SLICE_PAIRS_MAX || ld < n_pad || lda < n_pad ||
        n_pad % 16 || n < 1 || n > n_pad || n_pad >= (1 << 18))
        return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<int64_t>(n_pad, 16384);
    hipLaunchKernelGGL(slice_rows_kernel, dim3(grid), dim3(256), 0, s, U, ld, n_pad, n, S, A, lda, rscale, rsum);
    return hipGetLastError();
}

hipError_t snp_constants(const double* S, int64_t lds, int q1, int t, double* consts, int* fail,
                         hipStream_t s) {
    if (q1 < 1 || q1 > 19 || t < 1 || lds < q1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(snp_constants_kernel, dim3(1), dim3(64), 0, s, S, lds, q1, t, consts, fail);
    return hipGetLastError();
}

}  // namespace gwas
