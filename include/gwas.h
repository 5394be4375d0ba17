/*
 * gwas.h - C ABI of the MI355X library for the generalized least-squares
 * solves of a mixed-model genome-wide association study.
 *
 * For every SNP i the library computes (Eq. 1, Section 1)
 *
 *     b_i = (X_i^T M^-1 X_i)^-1 X_i^T M^-1 y,     X_i = [X_L | x_i],
 *
 * with M (n x n) symmetric positive definite, X_L (n x (p-1)) the covariates
 * shared by all SNPs, x_i (n) the dosages of SNP i and y (n) the phenotype
 * (t phenotype columns may share M and X_i).  It follows the restructured
 * algorithm of Section 2.1 (Algorithm 1) and its streamed form of Section 3
 * (Algorithm 2):
 *
 *   gwas_init          L L^T = M; Xbar_L = L^-1 X_L, ybar = L^-1 y;
 *                      S_TL = Xbar_L^T Xbar_L, bbar_T = Xbar_L^T ybar.
 *   gwas_stream_block  for a block of SNP columns X_blk:
 *                      Xbar_blk = L^-1 X_blk; per SNP S_BL = xbar^T Xbar_L,
 *                      S_BR = xbar^T xbar, bbar_B = xbar^T ybar; then the
 *                      p x p system S_i b_i = bbar_i by Cholesky.
 *   gwas_free          releases the context.
 *
 * Conventions
 *   - All matrices are column-major with an explicit leading dimension
 *     (ld >= rows).  SNP i of a block is the contiguous n-vector at
 *     XR + i*ldx.  b_i is the contiguous p-vector at b + i*ldb (for t > 1
 *     traits: t consecutive p-vectors, trait-major), with the SNP coefficient
 *     last (index p-1) and the X_L coefficients first, in X_L's column order.
 *   - Device memory means memory of the context's HIP device; host memory
 *     may be pageable or pinned (pinned host memory is used in place).
 *   - Functions return GWAS_OK (0) or a positive GWAS_E_* code; no C++
 *     exception crosses this interface.  Every call that takes a context
 *     returns GWAS_E_STATE for a NULL, freed or poisoned context.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Calls switch to the context's device while they run and restore the
 *     caller's current device before they return.
 */
#ifndef GWAS_H
#define GWAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define GWAS_OK            0
#define GWAS_E_INVALID     1   /* bad argument; nothing was touched          */
#define GWAS_E_NOT_SPD     2   /* M is not positive definite (gwas_info)     */
#define GWAS_E_RANK_XL     3   /* X_L^T M^-1 X_L not numerically positive
                                  definite (a Cholesky pivot <= 1e-10 times
                                  its diagonal entry): X_L rank deficient   */
#define GWAS_E_NO_DEVICE   4   /* no usable gfx950 device                    */
#define GWAS_E_HIP         5   /* HIP runtime error (gwas_last_error)        */
#define GWAS_E_OOM         6   /* device allocation failed                   */
#define GWAS_E_STATE       7   /* NULL, freed or poisoned context            */
#define GWAS_E_WORKSPACE   8   /* caller workspace smaller than required     */

/* ---- arithmetic of the per-block triangular solve ----------------------- */
#define GWAS_FP64          0   /* everything in float64                     */
#define GWAS_FP32_REFINE   1   /* L^-1 x_i on float32 matrix cores (float32
                                  sums over K in the default tile with int8
                                  dosages; the other tiles move them to
                                  float64 every 16 stages of K); the column
                                  sums, the SNP cross products and the p x p
                                  solve in float64 with two refinement
                                  steps                                      */
#define GWAS_BF16_REFINE   2   /* as above with bfloat16 operands           */
/*
 * Stated error of the two *_REFINE modes against the float64 path.  S_BL =
 * x_i^T M^-1 X_L and bbar_B = x_i^T M^-1 y are formed in float64 from
 * W = M^-1 [X_L | y], so S_i and bbar_i are float64-exact except for
 * S_BR = ||L^-1 x_i||^2, whose product runs in the reduced type.  The SNP
 * coefficient b_SNP = c_i / s_i (c_i exact) and var_i = 1 / s_i therefore
 * carry the relative error of s_i = S_BR - S_BL S_TL^-1 S_BL^T, which is at
 * most 16 u kappa_i with u = 2^-24 (float32) or 2^-8 (bfloat16) and
 * kappa_i = S_BR / s_i = 1 / (1 - R_i^2) >= 1 (R_i^2: whitened R^2 of x_i
 * on X_L); measured float32 values on the workloads are about 1e-7
 * (kappa_i <= 5).  The covariate coefficients change by |db_SNP| times
 * |S_TL^-1 S_BL^T|, so b_i is within 1e-8 normwise only where |b_SNP| is
 * small against ||b_i|| (as when the covariate effects dominate).  For
 * float64-grade results from int8 dosages use GWAS_INT8_SLICED.
 */
#define GWAS_INT8_SLICED   3   /* L^-1 held as `slices` int8 digits per entry
                                  with a power-of-two scale per row, digits
                                  in pairs (radix 127 inside a pair, 128
                                  between pairs); the product with int8
                                  dosages runs on int8 matrix cores with
                                  exact int32 sums and one float64
                                  combination; cross products and the p x p
                                  solve as in GWAS_FP32_REFINE.  Needs
                                  x_dtype = GWAS_X_I8 and n <= 260,096.
                                  The default tile shape adds both digits of
                                  a pair into one sum (the hi digit against
                                  127 (x - 1), in int8 only for dosages 0, 1
                                  or 2; the lo digit against x): a SNP with any other value gets NaN in
                                  b and var_snp (tile shape 0, through
                                  GWAS_TRMM_CFG or gwas_autotune, takes any
                                  int8 value).                            */

#define GWAS_BF16X3_REFINE 4  /* L^-1 held as three bfloat16 slices per
                                  entry (each rounds what the ones before it
                                  leave: their sum is L^-1 to about 2^-27
                                  relative); float64 dosages are cut into
                                  three slices the same way, once per
                                  sub-block before its product (3 n_pad x 2
                                  bytes of workspace per column), int8
                                  dosages are exact in bfloat16.  The
                                  products of slices i + j <= 2 (six; three
                                  with int8 dosages) run on bfloat16 matrix
                                  cores into the same float32 sums (float64
                                  every 16 stages of K in the tiles that keep
                                  float64 sums).  Cross products and the
                                  p x p solve as in GWAS_FP32_REFINE, with
                                  its stated error (u = 2^-24)           */

/* ---- element type of the SNP dosages handed to gwas_stream_block -------- */
#define GWAS_X_F64         0   /* float64                                   */
#define GWAS_X_I8          1   /* int8 dosages (0, 1, 2), expanded on device */

typedef struct gwas_ctx gwas_ctx;

typedef struct gwas_desc {
    int64_t n;               /* individuals, n >= p                          */
    int32_t p;               /* columns of X_i, 2 <= p <= 20                 */
    int32_t t;               /* phenotype columns sharing M, 1 <= t <= 256   */
    const double* M;         /* n x n, lower triangle read (Section 2)       */
    int64_t ldm;             /* >= n                                         */
    const double* XL;        /* n x (p-1) covariates                         */
    int64_t ldxl;            /* >= n                                         */
    const double* Y;         /* n x t phenotypes                             */
    int64_t ldy;             /* >= n                                         */
    int32_t inputs_on_device;/* nonzero: M, XL and Y are device pointers     */
    int32_t precision;       /* GWAS_FP64 | GWAS_FP32_REFINE | GWAS_BF16_REFINE
                                | GWAS_INT8_SLICED | GWAS_BF16X3_REFINE       */
    int32_t x_dtype;         /* GWAS_X_F64 | GWAS_X_I8                       */
    int32_t device;          /* HIP device ordinal                           */
    int64_t dev_block;       /* SNP columns per device sub-block, 0 = auto   */
    void*   workspace;       /* caller device memory, or NULL: library allocates */
    size_t  workspace_bytes; /* size of workspace when given                 */
    void*   stream;          /* hipStream_t the caller's inputs are produced on
                                (NULL = the default stream): every call first
                                waits for the work queued there; the library
                                computes on streams of its own            */
    int32_t slices;          /* GWAS_INT8_SLICED: digits per entry, 4..6
                                (0 = 6); ignored otherwise                  */
    int64_t band;            /* 0: M is dense (n x n, ldm >= n).  w >= 1: M is
                                banded, M(i,j) = 0 for |i - j| > w (relatives
                                grouped near the diagonal, Section 5.1), and
                                M holds its lower band in LAPACK band storage:
                                M(i,j) at M[(i - j) + j*ldm] for
                                j <= i <= min(n-1, j+w), ldm >= w+1.  Needs
                                GWAS_FP64; the factor is kept as blocks of
                                W = w rounded up to a multiple of 256 rows
                                (block bidiagonal) and each streamed block is
                                solved by block forward substitution, about
                                3 n W flops per SNP instead of n^2, for
                                n <= 2,000,000 with float64 dosages and
                                n <= 16,000,000 with int8.  With
                                int8 dosages and W <= 512 a sub-block walks
                                all block rows in one launch, Z on chip; else
                                (or with the environment variable
                                GWAS_BAND_STEP=1 at gwas_init, a measurement
                                and test aid) one launch per block row, with
                                the same results bit for bit.
                                gwas_stream_group, gwas_autotune,
                                gwas_stream_block_noalloc and the
                                gwas_backward_* calls return GWAS_E_INVALID
                                on such a context.                          */
} gwas_desc;

/*
 * Device bytes a context needs for these sizes (pure function, no device
 * call).  Returns 0 if the sizes are invalid.  A caller that passes its own
 * workspace must pass at least this many bytes, 256-byte aligned.
 */
size_t gwas_workspace_bytes(int64_t n, int32_t p, int32_t t, int64_t dev_block,
                            int32_t precision, int32_t x_dtype);   /* slices = 6 */

/*
 * Device bytes a context with a banded M (half-bandwidth band >= 1, band
 * storage with leading dimension ldm >= band + 1, GWAS_FP64) needs; 0 if
 * the sizes are invalid.  Pure function.
 */
size_t gwas_workspace_bytes_band(int64_t n, int32_t p, int32_t t, int64_t dev_block, int64_t band,
                                 int64_t ldm, int32_t x_dtype);

/*
 * Create a context: copies M, X_L and y to the device, factors M = L L^T
 * (Algorithm 1, first line; FP64), forms the explicit triangular inverse
 * L^-1 used by every block, whitens X_L and y (Algorithm 1, second line) and
 * forms S_TL, bbar_T and the Cholesky factor of S_TL (Algorithm 1, third
 * line).  For the GWAS_*_REFINE precisions it also forms
 * W = M^-1 [X_L | y] in float64 and the reduced-precision copy of L^-1.
 *
 * The desc's host pointers are only read during the call.  On success *out
 * owns all library memory (the caller's workspace, if given, must outlive
 * it).  Errors: GWAS_E_INVALID (n < p, p outside 2..20, t outside 1..256,
 * ld < n, NULL pointer, unknown precision or x_dtype; checked before any
 * device call; GWAS_INT8_SLICED with float64 dosages or slices outside
 * 4..6; band < 0, band > 0 with another precision than GWAS_FP64, or
 * ldm < band + 1), GWAS_E_NO_DEVICE, GWAS_E_WORKSPACE, GWAS_E_OOM, GWAS_E_HIP,
 * GWAS_E_NOT_SPD (gwas_info gives the 1-based order of the first leading
 * minor of M that is not positive, as LAPACK's potrf does) and
 * GWAS_E_RANK_XL.  On GWAS_E_NOT_SPD and GWAS_E_RANK_XL *out is set so that
 * gwas_info can be read, and must then be released with gwas_free; on every
 * other error *out is NULL.
 */
int gwas_init(gwas_ctx** out, const gwas_desc* d);

/*
 * Solve the GLS problems of a block of mblk SNPs (Algorithm 2, one pass of
 * its loop; the block is split into device sub-blocks of dev_block columns,
 * double-buffered between host-to-device copies and compute).
 *
 *   XR       n x mblk dosages (x_dtype), column i = SNP i, host or device.
 *            Device dosages are read in place when XR is 16-byte aligned
 *            and ldx spans a multiple of 16 bytes, at most 4 MiB; otherwise
 *            each sub-block is first copied into the library's buffer.
 *   ldx      >= n, elements between consecutive SNP columns.
 *   b        output, p*t doubles per SNP at b + i*ldb (host or device).
 *   ldb      >= p*t.
 *   var_snp  optional (NULL): [S_i^-1]_{pp}, the variance of the SNP
 *            coefficient in units of M, per SNP (host or device).
 *   info     optional (NULL): per-SNP status, 0 = solved, p = X_i
 *            numerically rank deficient (then b_i and var_i are NaN):
 *            s_i <= tol S_BR, i.e. the whitened R^2 of x_i on X_L is at
 *            least 1 - tol, with tol 1e-10 (GWAS_FP64, GWAS_INT8_SLICED),
 *            1e-6 (GWAS_FP32_REFINE, GWAS_BF16X3_REFINE) or 1e-2
 *            (GWAS_BF16_REFINE).  In the reduced modes this also flags SNPs
 *            too close to collinear for their product to resolve s_i.
 *
 * Returns after every output has been written (synchronous for the caller,
 * pipelined inside).  mblk = 0 is a no-op.  Results for a SNP do not depend
 * on the block it arrives in.  On a device error the context is poisoned and
 * later calls return GWAS_E_STATE; the work the failed call queued is
 * finished before it returns, so no copy into the caller's buffers is still
 * running.
 */
int gwas_stream_block(gwas_ctx* ctx, const void* XR, int64_t ldx, int64_t mblk,
                      double* b, int64_t ldb, double* var_snp, int32_t* info);

/*
 * Queue a block as gwas_stream_block does and return at once: Algorithm 2's
 * load and store of a block without their waits.  The block's copies in,
 * products, solves and copies out run on the context's streams behind the
 * blocks queued before it, so a caller that queues its blocks one after
 * another has the next block's copies overlap this block's products.  XR
 * must stay allocated and unchanged, and b, var_snp and info allocated and
 * untouched, until gwas_stream_wait returns.  Arguments and errors are
 * those of gwas_stream_block; a device error may surface here or in
 * gwas_stream_wait, and poisons the context.  Kernel timing
 * (gwas_set_timing) covers queued blocks too; their launches are counted
 * once they have been waited for.
 */
int gwas_stream_block_async(gwas_ctx* ctx, const void* XR, int64_t ldx, int64_t mblk,
                            double* b, int64_t ldb, double* var_snp, int32_t* info);

/*
 * Wait for every block gwas_stream_block_async queued on ctx; their outputs
 * are then written.  gwas_stream_block, gwas_stream_group, gwas_autotune and
 * the gwas_backward_* calls wait for queued blocks themselves.
 */
int gwas_stream_wait(gwas_ctx* ctx);

/*
 * For callers that cannot allocate memory or wait on the host: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same solves as gwas_stream_block, queued on the context's stream (the
 * desc's `stream`) behind the work queued there and on the context, and
 * returned from at once: the outputs are written when that stream reaches
 * this point.  The call allocates nothing (no hipMalloc, hipFree, pinned
 * memory or events) and copies nothing between host and device: XR (16-byte
 * aligned, ldx * element size a multiple of 16 and at most 4 MiB), b,
 * var_snp and info must all be device memory (GWAS_E_INVALID otherwise).
 * The per-SNP scratch of each sub-block (the product's partial sums, their
 * chunk totals, in the reduced modes the cross products x^T W and, in the
 * bfloat16 modes with float64 dosages, their cut bfloat16 copy) lives in
 * one static device buffer of 256 MiB that every GPU the library runs on
 * holds until the process ends; sub-blocks are as wide as fits it (at most
 * dev_block columns).  Every entry of it a call reads, that call writes
 * first, so nothing needs clearing between calls.  A context whose scratch
 * for 128 SNP columns exceeds 256 MiB (large n with many traits) gets
 * GWAS_E_INVALID, with the sizes in gwas_last_error.  Results equal gwas_stream_block's bit for bit.  All
 * contexts on one device share the buffer: calls that overlap in time on
 * one device (other streams, other contexts, other host threads) race and
 * must be ordered by the caller.  Kernel timing does not cover these calls.
 * Errors as gwas_stream_block.
 */
int gwas_stream_block_noalloc(gwas_ctx* ctx, const void* XR, int64_t ldx, int64_t mblk,
                              double* b, int64_t ldb, double* var_snp, int32_t* info);

/*
 * Several cohorts at once (the multi-cohort, multi-trait workload): contexts
 * with their own M, X_L, y and n, sharing the SNP positions of a block of
 * mblk SNPs.  Each sub-block of every context goes into ONE grouped launch
 * of the triangular product, whose tile schedule deals every (context, row
 * block) to the XCDs longest first, so cohorts of uneven n fill the chip
 * together; the cross products and p x p solves follow per context.
 * Each context's cross products, chunk sums and solves run on that
 * context's own stream after the product, so those of different contexts
 * overlap.  Results are identical to gwas_stream_block on each context.
 *
 *   ctxs, nctx   1..64 distinct contexts on one device with the same
 *                precision, x_dtype, dev_block and tile shape
 *   XR[i], ldx[i], b[i], ldb[i], var_snp[i], info[i]   as in
 *                gwas_stream_block for context i (var_snp, info and their
 *                entries may be NULL)
 *   flags        GWAS_GROUP_GRAPH: full-width sub-blocks replay one HIP
 *                graph of the grouped product, cross products and solves,
 *                captured at first use.  The product and the cross
 *                products read device dosages in place (the graph's
 *                argument array is updated before a replay when the
 *                pointers change); host dosages are copied into fixed
 *                device buffers; results are copied out of fixed buffers
 *
 * All work runs on the first context's compute stream; the call returns
 * when every output is written.  Errors: GWAS_E_INVALID (incompatible or
 * repeated contexts, bad sizes), GWAS_E_STATE, GWAS_E_HIP, GWAS_E_OOM.
 */
#define GWAS_GROUP_GRAPH 1
int gwas_stream_group(gwas_ctx* const* ctxs, int32_t nctx, const void* const* XR,
                      const int64_t* ldx, int64_t mblk, double* const* b, const int64_t* ldb,
                      double* const* var_snp, int32_t* const* info, int32_t flags);

/*
 * Pick the tile shape of the triangular product and the row-group size of
 * its XCD schedule (row tiles that share one L2: 1, 2, 4 or 8) by timing
 * every admissible pair on `cols` (<= dev_block) SNP columns of XR (host or
 * device), then, with that pair, the sub-block width gwas_stream_block
 * splits blocks into (dev_block, half or a quarter of it, those of whole
 * multiples of 128 columns that fit in `cols`), and keep the fastest for
 * later calls (gwas_query reports the width; gwas_stream_group keeps
 * dev_block).  With the environment
 * variable GWAS_TUNE_CACHE naming a file, an earlier result for the same
 * padded n, precision, dosage type and width is reused and new results are
 * appended.  *best_cfg (may be NULL) receives the chosen shape (for
 * GWAS_INT8_SLICED: 0 stages its operands through registers, 1 and 2 load
 * them straight into LDS, 2 with a wider tile; 3 to 5 add the two digits of
 * a pair into one sum against centred dosages, 3 staging through registers,
 * 4 to 6 loading straight into three or two LDS buffers, 6 (128-byte
 * stages) the default;
 * for GWAS_FP64, 7, the default, loads both operands straight into LDS,
 * int8 or float64 dosages); *best_rgroup (may be NULL) the row group.
 * For GWAS_FP64 and GWAS_INT8_SLICED, results of later calls are unchanged
 * up to float64 rounding order.  For the float32 and bfloat16 products a
 * shape also decides how their sums are kept: the 256 x 256 shape (6, the
 * default with int8 dosages) keeps float32 sums, the others move them to
 * float64 every 16 stages; b stays within the stated error of the *_REFINE
 * modes (16 u kappa_i on the SNP coefficient and var) either way.
 *
 * The environment variable GWAS_TRMM_CFG (read by gwas_init) overrides the
 * default shape with one the autotuner would try (0..7, 0..6 for
 * GWAS_INT8_SLICED; ignored when the shape does not apply to the precision
 * and dosage type): a measurement and test aid.
 */
int gwas_autotune(gwas_ctx* ctx, const void* XR, int64_t ldx, int64_t cols, int32_t* best_cfg,
                  int32_t* best_rgroup);

/*
 * Reverse mode (one trait, t = 1): the gradient of a scalar loss l(b, var)
 * over the GLS solutions of Eq. (1), given its cotangents gb_i = dl/db_i and
 * gv_i = dl/dvar_i.  With a_i = S_i^-1 gb_i, tau_i = S_i^-1 e_p,
 * Q_i = X_i^T M^-2 X_i and q_i = X_i^T M^-2 y (dM^-1 = -M^-1 dM M^-1):
 *   dl/dy        = M^-1 sum_i X_i a_i
 *   dl/dM        = Mbar = -sum_i sym(M^-1 X_i a_i (M^-1 (y - X_i b_i))^T)
 *                         + sum_i gv_i (M^-1 X_i tau_i)(M^-1 X_i tau_i)^T
 * and for a covariance model dM/dtheta = alpha M + beta I (for
 * M = sigma^2 (h^2 Phi + (1 - h^2) I): d/dh^2 has alpha = 1/h^2 and
 * beta = -sigma^2/h^2) the two contractions
 *   <Mbar, M> = sum_i gv_i var_i,
 *   tr Mbar   = sum_i [-a_i^T (q_i - Q_i b_i) + gv_i tau_i^T Q_i tau_i],
 * so that dl/dtheta = alpha <Mbar, M> + beta tr Mbar.  The per-SNP O(n^2)
 * work is one product w_i = M^-1 x_i (M^-1 = L^-T L^-1 formed once, float64).
 * Both contractions come back within about 1e-13 of the sum of the
 * magnitudes of their terms.  For d/dh^2 the two terms approach each other
 * as h^2 -> 0 (M -> sigma^2 I): the difference keeps their absolute errors,
 * so its relative error grows like (|<Mbar, M>| + sigma^2 |tr Mbar|) /
 * (h^2 |dl/dh^2|) times about 1e-14 (5e-11 measured at h^2 = 0.001).
 *
 *   gwas_backward_begin  forms M^-1 and W (first call allocates device
 *                        memory for them) and zeroes the accumulators.
 *   gwas_backward_block  one block: XR, ldx, mblk as given to
 *                        gwas_stream_block; b, ldb, var_snp, info its outputs;
 *                        gb (p per SNP, ldgb >= p) and gvar (NULL = 0) the
 *                        cotangents; host or device memory.  SNPs with
 *                        info != 0 contribute nothing.
 *   gwas_backward_end    gy (n doubles, host or device, may be NULL) = dl/dy,
 *                        *tr_mbar = tr Mbar, *ip_mbar_m = <Mbar, M>.
 * Errors: GWAS_E_INVALID (t != 1, bad sizes), GWAS_E_STATE (no begin),
 * GWAS_E_OOM, GWAS_E_HIP.
 */
int gwas_backward_begin(gwas_ctx* ctx);
int gwas_backward_block(gwas_ctx* ctx, const void* XR, int64_t ldx, int64_t mblk,
                        const double* b, int64_t ldb, const double* var_snp,
                        const int32_t* info, const double* gb, int64_t ldgb,
                        const double* gvar);
int gwas_backward_end(gwas_ctx* ctx, double* gy, double* tr_mbar, double* ip_mbar_m);

/*
 * Test hook for the error paths.  The k-th HIP status that later calls on
 * ctx check (k >= 1; 0 turns the hook off) is reported as failed
 * (hipErrorUnknown), as a real HIP error would be: that call returns
 * GWAS_E_HIP, the context is poisoned, gwas_last_error names the check and
 * ends in "(injected)", and the work the call had queued is finished before
 * it returns.  Nothing fails on the device.  Returns GWAS_E_STATE for a
 * NULL, freed or poisoned context and GWAS_E_INVALID for k < 0.
 */
int gwas_test_inject_fault(gwas_ctx* ctx, int64_t k);

/* Release a context (NULL is accepted).  Later use returns GWAS_E_STATE. */
int gwas_free(gwas_ctx* ctx);

/* Static text for a status code. */
const char* gwas_strerror(int code);

/* After GWAS_E_NOT_SPD: 1-based failing pivot of M; after GWAS_E_RANK_XL:
 * 1-based failing pivot of X_L^T M^-1 X_L; otherwise 0.  -1 for a bad ctx. */
int64_t gwas_info(const gwas_ctx* ctx);

/* Text of the last error recorded on the context ("" if none). */
const char* gwas_last_error(const gwas_ctx* ctx);

/*
 * Kernel timing for measurement: when enabled, HIP events bracket every
 * launch of the per-block triangular-product kernel on the compute stream
 * (synchronous and queued blocks, grouped launches).  gwas_kernel_time
 * returns the number of timed launches and their summed duration in
 * milliseconds since timing was last set, and the sum of the SNP columns
 * those launches processed; launches of queued blocks count once
 * gwas_stream_wait (or any call that waits for queued blocks) has returned.
 * gwas_set_timing first waits for queued blocks, which are timed under the
 * previous setting.
 */
int gwas_set_timing(gwas_ctx* ctx, int32_t enable);
int gwas_kernel_time(gwas_ctx* ctx, int64_t* launches, double* total_ms,
                     int64_t* columns);

/* Sizes of the context: n_pad (padded order of the device factors), the
 * sub-block width of gwas_stream_block (dev_block, or the width
 * gwas_autotune chose) and the device ordinal. */
int gwas_query(const gwas_ctx* ctx, int64_t* n_pad, int64_t* dev_block,
               int32_t* device);

/* ---- measured matrix-core peak ------------------------------------------
 * Sustained rate, in operations per second, of the matrix-core instruction
 * the triangular product of precision `kind` runs (GWAS_FP64: float64
 * 16x16x4; GWAS_FP32_REFINE: float32 16x16x4; GWAS_BF16_REFINE: bfloat16
 * 16x16x32; GWAS_INT8_SLICED: int8 16x16x64), on `device`, with `iters`
 * runs of 8 independent instructions per wave over a launch that fills the
 * chip (after an equal untimed launch that lets the clock settle).  It
 * measures the clock the device holds under matrix load, beside the
 * published peak that fractions of peak are quoted against.  Allocates and
 * frees a 4 MB device buffer; needs no context; leaves the current device
 * as it was.  GWAS_E_INVALID for a bad kind, iters outside [1, 2^32] or a
 * NULL result pointer; GWAS_E_NO_DEVICE, GWAS_E_OOM or GWAS_E_HIP. */
int gwas_peak_probe(int32_t kind, int32_t device, int64_t iters, double* ops_per_s);

#ifdef __cplusplus
}
#endif

#endif /* GWAS_H */
