// Internal declarations shared by the library's translation units.
// Launchers take raw device pointers and a stream; every launcher checks the
// shapes it is given against what its kernel assumes before launching.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "schedule.h"

namespace gwas {

// ---- tiles of the matrix-core kernels ----------------------------------
constexpr int TILE_M = 128;        // rows of a tile (rows of L^-1 / of C)
constexpr int TILE_N = 128;        // columns of a tile (SNPs / columns of C)
constexpr int NPAD_ALIGN = 256;    // n is padded to a multiple of this
constexpr int LEAF = 64;           // order of the diagonal blocks factored in LDS

// K-range restrictions of the generic FP64 product, from operand structure.
enum : int {
    KR_A_LOWER = 1,   // A(m,k) = 0 for k > m
    KR_A_UPPER = 2,   // A(m,k) = 0 for k < m
    KR_B_UPPER = 4,   // B(k,n) = 0 for k > n
    KR_B_LOWER = 8,   // B(k,n) = 0 for k < n
};

// C(MxN) = alpha * op(A) op(B) + beta * C in float64 on matrix cores.
//   opA 'N': A(m,k) = A[m + k*lda]      opA 'T': A(m,k) = A[k + m*lda]
//   opB 'N': B(k,n) = B[k + n*ldb]      opB 'T': B(k,n) = B[n + k*ldb]
// beta == 0 never reads C.  lower_only skips tiles strictly above the
// diagonal (for a symmetric update of a diagonal block).
struct GemmArgs {
    int64_t M, N, K;
    const double* A; int64_t lda; char opA;
    const double* B; int64_t ldb; char opB;
    double* C; int64_t ldc;
    double alpha, beta;
    int kflags;
    int lower_only;
};
hipError_t gemm_f64(const GemmArgs& g, hipStream_t s);

// Cholesky of the LEAF x LEAF diagonal block at L (lower triangle read),
// written back as L's block (zero above the diagonal) and the block of
// U = L^-T (zero below the diagonal).  Pivot failures of rows < n_valid
// record the smallest 1-based global row in *fail (atomic min).
hipError_t chol_leaf(double* L, double* U, int64_t ld, int64_t row0,
                     int64_t n_valid, int* fail, hipStream_t s);

// rows r >= n or columns c >= n of the n_pad x n_pad matrix A become identity
hipError_t pad_identity(double* A, int64_t ld, int64_t n, int64_t n_pad, hipStream_t s);

// out = (T)in over an n_pad x n_pad column-major block (same ld)
hipError_t convert_f32(const double* in, float* out, int64_t ld, int64_t rows,
                       int64_t cols, hipStream_t s);
hipError_t convert_bf16(const double* in, __bf16* out, int64_t ld, int64_t rows,
                        int64_t cols, hipStream_t s);

// Constant p x p blocks: S (q1 x Qc, ld lds) holds [S_TL | bbar_T] with
// q1 = p-1 rows.  Writes R = chol(S_TL) (lower, ld q1), v = R^-1 bbar_T
// (q1 x t), copies of S_TL and bbar_T, and the 1-based failing pivot of
// S_TL (0 if none) into *fail.
hipError_t snp_constants(const double* S, int64_t lds, int q1, int t,
                         double* consts, int* fail, hipStream_t s);

// Offsets into the constants buffer.
__host__ __device__ inline int64_t consts_R(int) { return 0; }
__host__ __device__ inline int64_t consts_v(int q1) { return (int64_t)q1 * q1; }
__host__ __device__ inline int64_t consts_STL(int q1, int t) { return (int64_t)q1 * q1 + (int64_t)q1 * t; }
__host__ __device__ inline int64_t consts_bT(int q1, int t) { return 2 * (int64_t)q1 * q1 + (int64_t)q1 * t; }
__host__ __device__ inline int64_t consts_len(int q1, int t) { return 2 * (int64_t)q1 * q1 + 2 * (int64_t)q1 * t; }

// ---- streaming kernels ---------------------------------------------------
// Dosage columns are read in place only with a column stride of at most this
// many bytes: a tile of up to 256 columns then spans less than 2^31 bytes,
// which the 32-bit offsets of the products' buffer loads need.  Wider
// strides go through the library's staging buffer.
constexpr int64_t X_DIRECT_MAX_LD_BYTES = int64_t(4) << 20;

enum AType : int { A_F64 = 0, A_F32 = 1, A_BF16 = 2, A_I8S = 3 };
// Dosage operand of the product: float64, int8, or float64 dosages cut once
// per sub-block into bfloat16 for the bfloat16 products: three slices of
// each column for the bfloat16-slice mode (X_BF16S, slice_x_bf16: slice i of
// column j at X + j*ldx + i*n_pad), one rounding for the bfloat16 mode
// (X_BF16, convert_x_bf16: column j at X + j*ldx); zero from row n on.
enum XType : int { X_F64 = 0, X_I8 = 1, X_BF16S = 2, X_BF16 = 3 };
inline int64_t x_elem_bytes(int xt) { return xt == X_I8 ? 1 : (xt == X_BF16S || xt == X_BF16) ? 2 : 8; }

// Z = L^-1 X for one sub-block, never stored: for every slice of part_rows
// rows of Z (one wave's rows) and SNP column j the kernel writes partial
// sums into
//   part[(pb * Q + q) * ldp + j]
// with q < Qc: z^T C[:,q] (only when with_cross) and q = Q-1: z^T z.
//   Ut    row-major L^-1 (Ut[k + r*ldu] = L^-1(r,k)), n_pad x n_pad, zero
//         above the diagonal and in the padding; element type per `at`.
//   X     n x cols dosages, column j at X + j*ldx (element type per `xt`).
//   C     n_pad x Qc whitened [Xbar_L | Ybar] (zero padding rows).
//   sched two int32 per workgroup: (row tile, column tile), -1 = idle.
//   cfg   tile shape (trmm_shape).
// Schedule entries: (row tile | context << SCHED_CTX_SHIFT, column tile).
constexpr int MAX_GROUP = 64;

struct TrmmArgs {
    int at, xt, cfg;
    const TrmmArgs* group;      // grouped launch: device array of per-context arguments
    int slices;                 // A_I8S: int8 slices per row of L^-1; A_BF16: 3 for the
                                // bfloat16-slice product (row r holds its slices one after
                                // another, n_pad elements each), else 0
    const double* rscale;       // A_I8S: power-of-two scale of each row of L^-1
    const int* rsum;            // A_I8S: rsum[p * n_pad + r] = sum over k < n of
                                // 127 A_2p(r, k), the hi digit of pair p
    const void* Ut; int64_t ldu; int64_t n_pad;
    const void* X; int64_t ldx; int64_t n; int64_t cols;
    const void* Xd; int64_t ldxd;  // the dosages as handed over (float64 or int8): X and ldx,
                                // or the float64 columns X_BF16S and X_BF16 are cut from
    const double* C; int64_t ldc; int Qc;
    int with_cross;
    double* part; int64_t ldp;
    const int* sched; int64_t n_sched;
    int full_k;                 // A is a full (not lower-triangular) n_pad x n_pad matrix
    int rgroup;                 // row tiles per L2 group of the schedule (0: the model's choice)
    int64_t sched_cols;         // columns the schedule was built for (0: cols); workgroups
                                // whose column tile starts at or past cols return at once
};
hipError_t trmm_stream(const TrmmArgs& a, hipStream_t s);
// the int8-slice kernel (a.at == A_I8S); called by trmm_stream
hipError_t trmm_sliced_launch(const TrmmArgs& a, hipStream_t s);
hipError_t trmm_check(const TrmmArgs& a, bool check_sched);

int trmm_num_cfgs();
int trmm_cfg_limit();              // one past the largest shape index of any product
bool trmm_shape_sum32(int cfg);   // shape keeps float32 sums only (reduced precision)
TrmmShape trmm_shape(int cfg);
bool trmm_cfg_valid(int at, int xt, int cfg);
int trmm_default_cfg(int at, int xt);
constexpr int MIN_PART_ROWS = 32;   // smallest part_rows of the floating-point shapes
// tiles of the int8-slice product (part_rows 16): shape cfg < trmm_sliced_cfgs()
int trmm_sliced_cfgs();
TrmmShape trmm_sliced_shape(int cfg = 0);
bool trmm_sliced_direct(int cfg);    // the shape loads its operands straight into LDS
bool trmm_sliced_paired(int cfg);    // the shape pairs digits against centred dosages
                                     // (dosages must be 0, 1 or 2)
bool trmm_sliced_two_per_cu(int cfg); // the shape runs two workgroups per CU
int trmm_sliced_default_cfg();        // the int8-slice shape used unless tuned
// shape of the kernel that runs (at, xt, cfg, slices), with its schedule
// grouping: rgroup row tiles per group, or the traffic model's choice for 0
TrmmShape trmm_geom(int at, int xt, int cfg, int slices, int rgroup = 0);
constexpr int RGROUP_CANDIDATES[] = {1, 2, 4, 8};   // what the autotuner tries

// Row r of L^-1 (column r of U, U[k + r*ld]) as three bfloat16 slices
// out[k + i*n_pad + r*ldo], i = 0..2 (ldo >= 3 n_pad): slice i rounds what
// slices 0..i-1 leave, so their sum is L^-1(r, k) to about 2^-27 relative.
hipError_t slice_bf16(const double* U, int64_t ld, int64_t n_pad, __bf16* out, int64_t ldo, hipStream_t s);
// The same cut for cols float64 dosage columns (column j at X + j*ldx,
// elements k < n): out[k + i*n_pad + j*ldo], i = 0..2, zero for n <= k < n_pad.
// With xargs (a device argument record) X and ldx are read from its Xd and
// ldxd when the kernel runs.
hipError_t slice_x_bf16(const double* X, int64_t ldx, int64_t n, int64_t n_pad, int64_t cols, __bf16* out,
                        int64_t ldo, hipStream_t s, const TrmmArgs* xargs = nullptr);
// Float64 dosage columns rounded to bfloat16 (through float32, as the
// bfloat16 product's staging rounds them): out[k + j*ldo], zero for
// n <= k < n_pad; xargs as for slice_x_bf16.
hipError_t convert_x_bf16(const double* X, int64_t ldx, int64_t n, int64_t n_pad, int64_t cols, __bf16* out,
                          int64_t ldo, hipStream_t s, const TrmmArgs* xargs = nullptr);

// Row r of L^-1 (column r of U, U[k + r*ld]) -> rscale[r] = 2^e >= max |L^-1(r,k)|
// and S int8 digits A_s(r,k) in [-64, 64], written to sliced row
// (r/16)*16*S + s*16 + r%16 of A (lda bytes per row).  Digits come in pairs
// (hi A_2p, lo A_2p+1) with a radix of 127 inside a pair and 128 between
// pairs:  L^-1(r,k)/rscale[r] = sum_p D_p(r,k) w_p up to half a unit of the
// last digit, D_p = 127 A_2p + A_2p+1 (A_S = 0 for odd S) and
// w_p = 2^(-6-7p) / 127^(2p+1).  rsum[p * n_pad + r] = 127 sum_{k < n} A_2p(r,k).
constexpr int SLICE_PAIRS_MAX = 3;
hipError_t slice_rows(const double* U, int64_t ld, int64_t n_pad, int64_t n, int S, int8_t* A,
                      int64_t lda, double* rscale, int* rsum, hipStream_t s);

// Host side: tile schedule for n_pad rows and `cols` SNP columns with the
// tiles of `sh`.  Returns the number of workgroups and fills `out` (2 ints
// each; -1 = idle workgroup).  The multi-context form takes each context's
// row-tile count and tags entries with the context index.
int64_t trmm_schedule(int64_t n_pad, int64_t cols, const TrmmShape& sh, int* out, int64_t cap);
int64_t trmm_schedule_len(int64_t n_pad, int64_t cols, const TrmmShape& sh);
// (trmm_schedule_multi, the multi-context form, is in schedule.h)

// xw[q * ldxw + j] = x_j^T W[:, q] for q < Qc (float64 matrix cores).  W has
// ldw >= n rounded up to 16 rows, zero past n.  With part (room for
// part_cap doubles, at least xw_splits(n) * Qc * cols) K is split in chunks
// fixed by n and the partial sums are added in order; without it, one split.
// check012 (int8 dosages): a SNP with a dosage outside {0, 1, 2} gets NaN.
// xargs (device memory, may be null): the kernel takes X and ldx from
// xargs->X and xargs->ldx when it runs (X and ldx here are only checked).
int xw_splits(int64_t n);
hipError_t snp_cross_w(int xt, const void* X, int64_t ldx, int64_t n, int64_t cols,
                       const double* W, int64_t ldw, int Qc, double* xw,
                       int64_t ldxw, double* part, int64_t part_cap, hipStream_t s,
                       bool check012 = false, const TrmmArgs* xargs = nullptr);

// Reverse mode through the per-SNP solves (one trait).  For SNP j, with the
// Cholesky factor of S_j from R = chol(S_TL), S_BL = x^T W_L and s = 1/var,
// and the cotangents gb (p values) and gv of b_j and var_j:
//   a = S^-1 gb, tau = S^-1 e_p;  Q = X^T M^-2 X and q = X^T M^-2 y from
//   G = W_L^T W_L, gy0 = W_L^T w_y (constants) and the partial sums of
//   w = M^-1 x against [W_L | w_y] and w^T w (part, Q = p+1 rows per slice);
// writes contrib[k*ldc + j]: k < p-1: a_L; k = p-1: -a^T (q - Q b) + gv tau^T Q tau;
// k = p: gv var; and coef[j] = a_SNP (SNPs with info != 0 contribute zero).
struct BackArgs {
    int p;
    int64_t cols;
    const double* part; int64_t ldp; int64_t npb;   // partials of the M^-1 product
    const double* xw; int64_t ldxw;                 // x^T [W_L | w_y]
    const double* consts;                           // R (as in snp_constants)
    const double* G; const double* gy0;             // W_L^T W_L ((p-1)^2), W_L^T w_y (p-1)
    const double* b; int64_t ldb; const double* var; const int* info;
    const double* gb; int64_t ldgb; const double* gv;
    double* contrib; int64_t ldc;
    double* coef;
};
hipError_t snp_backward(const BackArgs& a, hipStream_t s);

// One block row of the banded forward substitution for every SNP column of
// a sub-block: Z_i = U_ii^T X_i + Gt^T Z_{i-1} (W x cols, float64), stored
// into Zcur (column j at Zcur + j*ldz), with the partial sums of the dense
// product (part[(pb*Q + q)*ldp + j], Q = Qc + 1, pb = global 32-row slice:
// z^T C[:,q] for q < Qc and z^T z).
//   Ut   U_ii = L_ii^-T, W x W column-major (row r of L_ii^-1 at Ut + r*W)
//   Gt   -E_i^T U_ii (W x W column-major; unused in block row 0)
//   X    n x cols dosages (xt), column j at X + j*ldx; rows blk*W.. are X_i
//   C    n_pad x Qc whitened [Xbar_L | Ybar], ld ldc
struct BandArgs {
    int xt;
    int64_t W, blk, nb;           // block order, block row (band_step), block rows (band_walk)
    const double* Ut; const double* Gt;
    const void* X; int64_t ldx; int64_t n; int64_t cols;
    const double* Zprev; double* Zcur; int64_t ldz;
    const double* C; int64_t ldc; int Qc;
    double* part; int64_t ldp;
};
hipError_t band_step(const BandArgs& a, hipStream_t s);
int band_part_rows();   // rows per partial-sum slice of band_step and band_walk (32)
// All nb block rows of a sub-block in one launch (int8 dosages, W of 256 or
// 512: band_walk_fits): Ut and Gt point at block row 0's U_00 and Gt_0, Z
// stays on chip (Zprev, Zcur unused); the same partial sums as nb calls of
// band_step.
bool band_walk_fits(int xt, int64_t W);
hipError_t band_walk(const BandArgs& a, hipStream_t s);
// out (rows x cols, ld ldo) = block (row0.., col0..) of the SPD M given in
// LAPACK lower band storage of half-bandwidth w (M(i,j) at AB[(i-j) + j*ldab],
// j <= i <= j + w); zero above the diagonal and outside the band, identity
// past n.
hipError_t band_block(const double* AB, int64_t ldab, int64_t w, int64_t n, int64_t row0, int64_t col0,
                      int64_t rows, int64_t cols, double* out, int64_t ldo, hipStream_t s);

// Partial sums of the triangular product reduced in chunks of `chunk`
// slices: out[(g*Q + q)*ldo + j] = sum over pb in chunk g (ascending) of
// part[(pb*Q + q)*ldp + j], for g < ceil(npb / chunk).  The per-SNP kernels
// then sum the few chunk totals; the order depends on npb (n) alone.
constexpr int PART_CHUNK = 32;
hipError_t partial_chunks(const double* part, int64_t ldp, int64_t npb, int Q, int64_t cols, int chunk,
                          double* out, int64_t ldo, hipStream_t s);
inline int64_t chunks_of(int64_t npb) { return (npb + PART_CHUNK - 1) / PART_CHUNK; }

// acc[k] += sum_j contrib[k*ldc + j] for k < rows (fixed summation order).
hipError_t sum_columns(const double* contrib, int64_t ldc, int rows, int64_t cols, double* acc,
                       hipStream_t s);

// g[r] += sum_j X(r, j) coef[j] for r < n (dosages column-major, fixed order).
hipError_t dosage_gemv(int xt, const void* X, int64_t ldx, int64_t n, int64_t cols,
                       const double* coef, double* g, hipStream_t s);

// Per-SNP reduction of the partials and the p x p Cholesky solve.
struct SolveArgs {
    int p, t;
    int64_t cols;
    const double* part; int64_t ldp; int64_t npb; int Q;  // partials
    const double* xw; int64_t ldxw;                       // NULL: cross terms from part
    const double* consts;
    int refine;                                           // FP64 refinement steps
    double rank_tol;
    double* b; int64_t ldb;
    double* var;
    int* info;
};
hipError_t snp_solve(const SolveArgs& a, hipStream_t s);

}  // namespace gwas
