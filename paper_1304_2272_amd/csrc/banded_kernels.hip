// The per-block triangular solve for a banded M (the banded-matrix variant
// the paper names as future work, Section 5.1).  With M = L L^T of
// half-bandwidth w and blocks of W >= w rows, M is block tridiagonal and L
// block lower bidiagonal: L_ii on the diagonal and E_i = L_{i,i-1} below it.
// Forward substitution then runs block row by block row,
//     Z_i = L_ii^-1 (X_i - E_i Z_{i-1}) = U_ii^T X_i + Gt_i^T Z_{i-1},
// with U_ii = L_ii^-T and Gt_i = -E_i^T U_ii formed at set-up.  One launch
// of band_lds_kernel is one block row for every SNP column of a sub-block:
// a float64 matrix-core product with K = [the triangular part of U_ii^T |
// all of Gt_i^T] against [X_i | Z_{i-1}], which stores Z_i for the next
// block row and writes the same partial sums as the dense product (S_BL,
// bbar_B and S_BR of Algorithm 2 per 32-row slice of Z).
#include "internal.h"
#include "trmm_common.h"

#include <algorithm>

namespace gwas {
namespace {

constexpr int BT_M = 128, BT_N = 128, BT_NT = 512;   // tile and threads
constexpr int BT_WTM = 2, BT_WTN = 4;                 // 16 x 16 blocks per wave (32 x 64)
constexpr int BT_WGN = 2;                             // waves along the columns
constexpr int BT_BK = 16;                             // K per stage (one 128-byte row of doubles)
constexpr int BT_ROWS = BT_WTM * 16;                  // rows of a partial-sum slice

// One BT_M x BT_N tile of Z_i per workgroup, stages of 16 K, its operands
// loaded straight from global memory into two LDS buffers (the loads of
// stage s + 1 issued at the top of stage s, explicit waits and a bare
// barrier at its end), so no staging registers or LDS writes are spent on
// them and two workgroups share a CU.  Within a stage lane group g = lane/16
// supplies the contiguous K slice [4g, 4g + 4) to both operands, one K per
// instruction (the 16x16x4 float64 instruction sums its K in any order the
// two operands agree on).  Workgroup b runs on XCD b % 8: the row tiles of a
// column tile run on one XCD, so its dosage and Z panels stay in that L2.
// Rows of U_ii^T and Gt_i^T sit unpadded in 8-row groups of 128-byte stage
// rows, chunk c (16 bytes) of row r8 of a group in slot
// 16 (c / 2) + 8 ((c % 2) xor (group parity)) + r8, so a fragment read (16
// rows, one chunk) hits distinct banks whether the LDS serves 8 or 16 lanes
// of a 16-byte read per cycle; Z_{i-1} and float64 dosages sit in the same
// layout, int8 dosages as bytes (16 per column and stage, widened per
// fragment).  Int8 dosage bytes past n belong to the next column: they meet
// zeros of U_ii^T in every row below n, and the rows at or past n (only in
// the last block row, whose Z no block row reads) are zeroed before the
// sums; float64 dosages at or past n are read as zero, since the stride's
// padding may hold anything (NaN included).
template <typename XT>
__global__ __launch_bounds__(BT_NT, 4) void band_lds_kernel(BandArgs a) {
    constexpr bool XD = sizeof(XT) == 8;          // float64 dosages: laid out as the rows
    constexpr int WTM = BT_WTM, WTN = BT_WTN, NW = 8;
    constexpr int AB = BT_M * BT_BK * 8;          // bytes of U_ii^T or Gt_i^T per stage
    constexpr int ZB = BT_N * BT_BK * 8;          // bytes of Z_{i-1} per stage (dosages: the first 2 KB)
    constexpr int WAIT_ALL = 7 << 4;              // vmcnt(0) lgkmcnt(0)
    const int b = blockIdx.x;
    const int rtiles = (int)(a.W / BT_M);
    const int q0 = b >> 3;
    const int64_t ct = (b & 7) + 8 * (int64_t)(q0 / rtiles);
    const int rt = q0 % rtiles;
    const int64_t c0 = ct * BT_N;
    if (c0 >= a.cols) return;
    const int64_t r0 = (int64_t)rt * BT_M;
    const int64_t g0 = a.blk * a.W;

    __shared__ __attribute__((aligned(1024))) char Abuf[2][AB];
    __shared__ __attribute__((aligned(1024))) char Bbuf[2][ZB];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave / BT_WGN, wc = wave % BT_WGN;
    const int li = lane & 15, lg = lane >> 4;

    const int nA = (int)(std::min<int64_t>(r0 + BT_M, a.W) / BT_BK);
    const int nst = nA + (a.blk > 0 ? (int)(a.W / BT_BK) : 0);
    const int64_t row_bytes = a.W * 8;
    const u4_t rsU = buffer_words(a.Ut + r0 * a.W, (uint32_t)(BT_M * row_bytes));
    const u4_t rsG = a.blk > 0 ? buffer_words(a.Gt + r0 * a.W, (uint32_t)(BT_M * row_bytes)) : rsU;
    const int64_t xcols = std::min<int64_t>(BT_N, a.cols - c0);
    const u4_t rsX = buffer_words(static_cast<const char*>(a.X) + c0 * a.ldx * (int64_t)sizeof(XT),
                                  (uint32_t)((((xcols - 1) * a.ldx + a.n) * (int64_t)sizeof(XT) + 15) / 16 * 16));
    const u4_t rsZ = a.blk > 0 ? buffer_words(a.Zprev + c0 * a.ldz, (uint32_t)(xcols * a.ldz * 8)) : rsX;
    // lane l of a load of 8 rows fetches the chunk that belongs in slot l;
    // lane l of a dosage load, column l of its 64
    const int lr8 = lane & 7;
    const int lc_even = 2 * (lane >> 4) + ((lane >> 3) & 1);
    const int lc_odd = 2 * (lane >> 4) + (((lane >> 3) & 1) ^ 1);
    auto load = [&](int s, char* Ab, char* Bb) {
        const bool pu = s < nA;
        const int k0 = (pu ? s : s - nA) * BT_BK;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int q = wave + c * NW;
            const int ch = (q & 1) ? lc_odd : lc_even;
            load_lds16(pu ? rsU : rsG, lds_address(Ab + q * 1024),
                       (uint32_t)((q * 8 + lr8) * row_bytes + k0 * 8 + ch * 16));
        }
        if (pu && !XD) {
            if (wave < 2)
                load_lds16(rsX, lds_address(Bb + wave * 1024),
                           (uint32_t)((wave * 64 + lane) * a.ldx + g0 + k0));
        } else if (pu) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int q = wave + c * NW;
                const int ch = (q & 1) ? lc_odd : lc_even;
                load_lds16(rsX, lds_address(Bb + q * 1024),
                           (uint32_t)((q * 8 + lr8) * a.ldx * 8 + (g0 + k0) * 8 + ch * 16));
            }
        } else {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int q = wave + c * NW;
                const int ch = (q & 1) ? lc_odd : lc_even;
                load_lds16(rsZ, lds_address(Bb + q * 1024), (uint32_t)((q * 8 + lr8) * a.ldz * 8 + k0 * 8 + ch * 16));
            }
        }
    };

    d4_t acc[WTM][WTN];
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
    // this lane's fragment offsets in a stage buffer: rows wr*32 + i*16 + li,
    // chunks 2 lg + h, in the slots above; the group parity is that of li / 8
    // for every i, so
    // fragment i (column block j of Z_{i-1}) sits 2048 i (2048 j) bytes on
    // from fragment 0
    const int p8 = (li >> 3) & 1;
    const int lbase = (li >> 3) * 1024 + lg * 256 + (li & 7) * 16;
    const int abase = wr * WTM * 16 / 8 * 1024 + lbase;
    const int zbase = wc * WTN * 16 / 8 * 1024 + lbase;
    auto aoff = [&](int i, int h) { return abase + i * 2048 + ((h ^ p8) << 7); };
    auto zoff = [&](int j, int h) { return zbase + j * 2048 + ((h ^ p8) << 7); };
    const int xoff = (wc * WTN * 16 + li) * BT_BK + lg * 4;

    // the end of every stage: its matrix instructions stay ahead of the
    // barrier; this wave's loads of the next stage have landed, and after
    // the barrier every wave's have, and every wave is done with this one
    auto stage_end = [&]() {
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(WAIT_ALL);
        compiler_fence();
        __builtin_amdgcn_s_barrier();
        compiler_fence();
    };
    auto read_a = [&](const char* Ar, u4_t (&fa)[WTM][2]) {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int h = 0; h < 2; ++h) fa[i][h] = *reinterpret_cast<const u4_t*>(Ar + aoff(i, h));
    };
    auto a_val = [&](const u4_t (&fa)[WTM][2], int i, int e) {
        const u2_t w2 = (e & 1) ? u2_t{fa[i][e >> 1][2], fa[i][e >> 1][3]} : u2_t{fa[i][e >> 1][0], fa[i][e >> 1][1]};
        return __builtin_bit_cast(double, w2);
    };
    // the products of a stage whose B side holds float64 values in the
    // layout of the rows (Z_{i-1}, or float64 dosages), one 16-byte piece
    // (two K) of each fragment at a time
    auto stage_b64 = [&](const u4_t (&fa)[WTM][2], const char* Br) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            u4_t fz[WTN];
#pragma unroll
            for (int j = 0; j < WTN; ++j) fz[j] = *reinterpret_cast<const u4_t*>(Br + zoff(j, h));
#pragma unroll
            for (int e2 = 0; e2 < 2; ++e2) {
                const int e = 2 * h + e2;
                double zb[WTN];
#pragma unroll
                for (int j = 0; j < WTN; ++j)
                    zb[j] = __builtin_bit_cast(double, e2 ? u2_t{fz[j][2], fz[j][3]} : u2_t{fz[j][0], fz[j][1]});
#pragma unroll
                for (int i = 0; i < WTM; ++i) {
                    const double av = a_val(fa, i, e);
#pragma unroll
                    for (int j = 0; j < WTN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, zb[j], acc[i][j], 0, 0, 0);
                }
            }
        }
    };
    // a stage of the U_ii^T part: dosage bytes widened per fragment, or
    // float64 dosages in the layout of the rows with K at or past n read as
    // zero (the bytes past a column's n belong to whatever follows it)
    auto stage_u = [&](int s, const char* Ar, const char* Br, char* An, char* Bn) {
        if (s + 1 < nst) load(s + 1, An, Bn);
        u4_t fa[WTM][2];
        read_a(Ar, fa);
        if constexpr (XD) {
            // 8 bytes of a fragment at a time, K at or past n read as zero
            const int kl = (int)std::min<int64_t>(a.n - (g0 + s * BT_BK), BT_BK) - 4 * lg;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double xb[WTN];
#pragma unroll
                for (int j = 0; j < WTN; ++j) {
                    const double v = *reinterpret_cast<const double*>(Br + zoff(j, e >> 1) + (e & 1) * 8);
                    xb[j] = e < kl ? v : 0.0;
                }
#pragma unroll
                for (int i = 0; i < WTM; ++i) {
                    const double av = a_val(fa, i, e);
#pragma unroll
                    for (int j = 0; j < WTN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xb[j], acc[i][j], 0, 0, 0);
                }
            }
            stage_end();
            return;
        }
        uint32_t fb[WTN];
#pragma unroll
        for (int j = 0; j < WTN; ++j) fb[j] = *reinterpret_cast<const uint32_t*>(Br + xoff + j * 16 * BT_BK);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            double xb[WTN];
#pragma unroll
            for (int j = 0; j < WTN; ++j) xb[j] = (double)(int)(int8_t)(fb[j] >> (8 * e));
#pragma unroll
            for (int i = 0; i < WTM; ++i) {
                const double av = a_val(fa, i, e);
#pragma unroll
                for (int j = 0; j < WTN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xb[j], acc[i][j], 0, 0, 0);
            }
        }
        stage_end();
    };
    // a stage of the Gt_i^T part: Z_{i-1} in the layout of the rows
    auto stage_g = [&](int s, const char* Ar, const char* Br, char* An, char* Bn) {
        if (s + 1 < nst) load(s + 1, An, Bn);
        u4_t fa[WTM][2];
        read_a(Ar, fa);
        stage_b64(fa, Br);
        stage_end();
    };

    load(0, Abuf[0], Bbuf[0]);
    __builtin_amdgcn_s_waitcnt(WAIT_ALL);
    compiler_fence();
    __builtin_amdgcn_s_barrier();
    compiler_fence();
    // both parts have an even number of stages (nA a multiple of 8, W / 16
    // even), so each starts in buffer 0
    for (int s = 0; s < nA; s += 2) {
        stage_u(s, Abuf[0], Bbuf[0], Abuf[1], Bbuf[1]);
        stage_u(s + 1, Abuf[1], Bbuf[1], Abuf[0], Bbuf[0]);
    }
    for (int s = nA; s < nst; s += 2) {
        stage_g(s, Abuf[0], Bbuf[0], Abuf[1], Bbuf[1]);
        stage_g(s + 1, Abuf[1], Bbuf[1], Abuf[0], Bbuf[0]);
    }

    // Epilogue.  Element v of accumulator (i, j) holds row
    // r0 + wr*32 + i*16 + lg + 4v and column c0 + wc*64 + j*16 + li; rows at
    // or past n are zeroed first
    const int64_t rw = r0 + wr * BT_ROWS;
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (g0 + rw + i * 16 + lg + 4 * v >= a.n)
#pragma unroll
                for (int j = 0; j < WTN; ++j) acc[i][j][v] = 0.0;
    const int64_t pb = (g0 + rw) / BT_ROWS;
    const int64_t cbase = c0 + wc * BT_WTN * 16 + li;
    const int Q = a.Qc + 1;
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
        const int64_t col = cbase + j * 16;
        if (col < a.cols) {
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) a.Zcur[col * a.ldz + rw + i * 16 + lg + 4 * v] = acc[i][j][v];
        }
    }
    for (int qq = 0; qq < a.Qc; ++qq) {
        const double* Cq = a.C + qq * a.ldc + g0 + rw + lg;
        double cv[WTM][4];
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) cv[i][v] = Cq[i * 16 + 4 * v];
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
            double sum = 0.0;
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) sum += acc[i][j][v] * cv[i][v];
            sum = wave_sum16(sum);
            const int64_t col = cbase + j * 16;
            if (lg == 0 && col < a.cols) a.part[(pb * Q + qq) * a.ldp + col] = sum;
        }
    }
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) sum += acc[i][j][v] * acc[i][j][v];
        sum = wave_sum16(sum);
        const int64_t col = cbase + j * 16;
        if (lg == 0 && col < a.cols) a.part[(pb * Q + Q - 1) * a.ldp + col] = sum;
    }
}

// The whole block forward substitution of a sub-block in one launch, for
// int8 dosages and blocks of W = 128 WTM rows (256 or 512).  Workgroup b
// owns SNP columns [b TN, (b + 1) TN) and walks every block row; Z_{i-1} of
// its columns stays in LDS as float64 from one block row to the next, and
// the dosages of the block row sit there as bytes.  Wave w holds 16 WTM rows
// of Z_i and streams the same rows of U_ii^T and Gt_i^T from global memory
// (every workgroup reads the same block, so they come from L2) straight into
// registers, one stage ahead: rows are not shared between waves, so inside
// a block row no wave waits for another.  Two barriers per block row hand
// Z_i over.  The waves of a workgroup are dealt to the four SIMDs in turn,
// so waves w and w + 4 share one; they take row slices w and 7 - w, and
// each SIMD gets the same share of the triangular U_ii^T part.
// Per accumulator the matrix instructions, their K order (the triangular
// part up to the wave's last row, then all of Gt_i^T) and the partial sums
// per 32-row slice are those of band_lds_kernel; the stages it runs past a
// wave's last row multiply zeros of U_ii^T, so both kernels give the same
// values.  MINW waves per SIMD: 4 for two workgroups per CU.
template <int WTM, int WTN, int MINW>
__global__ __launch_bounds__(512, MINW) void band_walk_kernel(BandArgs a) {
    constexpr int NW = 8, RW = 16 * WTM, W = NW * RW, TN = 16 * WTN;
    constexpr int ZS = W * 8 + 16;            // bytes per Z column in LDS
    constexpr int XS = W + 16;                // bytes per dosage column in LDS
    constexpr int XCH = TN * W / 16;          // 16-byte dosage chunks of a block row
    constexpr int XPT = (XCH + 511) / 512;    // ... per thread
    constexpr int NG = W / 16;                // stages of the Gt_i^T part
    static_assert(WTM % 2 == 0, "32-row partial-sum slices");
    __shared__ __attribute__((aligned(16))) char Zs[TN * ZS];
    __shared__ __attribute__((aligned(16))) char Xs[TN * XS];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int rb = (wave < 4 ? wave : 11 - wave) * RW;   // first row of this wave in a block
    const int nU = rb / 16 + WTM;                          // stages of the U_ii^T part
    const int64_t c0 = (int64_t)blockIdx.x * TN;
    const int8_t* X = static_cast<const int8_t*>(a.X);
    const int64_t WW = (int64_t)W * W;

    // this thread's dosage chunks of block row i (zero past n and past the
    // sub-block), loaded a block row ahead and held in registers while the
    // block row before is done (XPRE), or, with the wave's 96 or 128 rows
    // taking the registers, loaded when the block row before is done (its
    // time then dwarfs the one wait)
    constexpr bool XPRE = WTM <= 4;
    u4_t xr[XPT];
    auto xload = [&](int64_t i) {
#pragma unroll
        for (int c = 0; c < XPT; ++c) {
            const int q = tid + 512 * c;
            xr[c] = u4_t{0u, 0u, 0u, 0u};
            if (XCH % 512 == 0 || q < XCH) {
                const int64_t col = c0 + q / (W / 16);
                const int64_t g = i * W + (q % (W / 16)) * 16;
                if (col < a.cols) {
                    const int8_t* src = X + col * a.ldx + g;
                    if (g + 16 <= a.n) {
                        xr[c] = *reinterpret_cast<const u4_t*>(src);
                    } else {
                        int8_t tmp[16] __attribute__((aligned(16)));
#pragma unroll
                        for (int e = 0; e < 16; ++e) tmp[e] = g + e < a.n ? src[e] : (int8_t)0;
                        xr[c] = *reinterpret_cast<const u4_t*>(tmp);
                    }
                }
            }
        }
    };
    auto xstore = [&]() {
#pragma unroll
        for (int c = 0; c < XPT; ++c) {
            const int q = tid + 512 * c;
            if (XCH % 512 == 0 || q < XCH)
                *reinterpret_cast<u4_t*>(Xs + (q / (W / 16)) * XS + (q % (W / 16)) * 16) = xr[c];
        }
    };
    // a lane's 4 doubles of K (4 lg ..) of its row in each 16-row fragment:
    // stage s of block row i, of U_ii^T for s < nU, else of Gt_i^T
    auto aload = [&](u4_t (&r)[WTM][2], int64_t i, int s) {
        const bool pu = s < nU;
        const double* base = (pu ? a.Ut : a.Gt) + i * WW + (int64_t)(rb + li) * W + 16 * (pu ? s : s - nU) + 4 * lg;
#pragma unroll
        for (int f = 0; f < WTM; ++f) {
            r[f][0] = *reinterpret_cast<const u4_t*>(base + f * 16 * W);
            r[f][1] = *reinterpret_cast<const u4_t*>(base + f * 16 * W + 2);
        }
    };

    d4_t acc[WTM][WTN];
#pragma unroll
    for (int f = 0; f < WTM; ++f)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[f][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    auto stage = [&](const u4_t (&r)[WTM][2], int s) {
        double fa[WTM][4];
#pragma unroll
        for (int f = 0; f < WTM; ++f) {
            fa[f][0] = __builtin_bit_cast(double, u2_t{r[f][0][0], r[f][0][1]});
            fa[f][1] = __builtin_bit_cast(double, u2_t{r[f][0][2], r[f][0][3]});
            fa[f][2] = __builtin_bit_cast(double, u2_t{r[f][1][0], r[f][1][1]});
            fa[f][3] = __builtin_bit_cast(double, u2_t{r[f][1][2], r[f][1][3]});
        }
        if (s < nU) {
            // dosages of columns j*16 + li, K = 16 s + 4 lg + e
            uint32_t fb[WTN];
#pragma unroll
            for (int j = 0; j < WTN; ++j)
                fb[j] = *reinterpret_cast<const uint32_t*>(Xs + (j * 16 + li) * XS + 16 * s + 4 * lg);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double xb[WTN];
#pragma unroll
                for (int j = 0; j < WTN; ++j) xb[j] = (double)(int)(int8_t)(fb[j] >> (8 * e));
#pragma unroll
                for (int f = 0; f < WTM; ++f)
#pragma unroll
                    for (int j = 0; j < WTN; ++j)
                        acc[f][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[f][e], xb[j], acc[f][j], 0, 0, 0);
            }
        } else {
            // Z_{i-1} of columns j*16 + li, K = 16 (s - nU) + 4 lg + e
            double zb[WTN][4];
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
                const char* p = Zs + (j * 16 + li) * ZS + (16 * (s - nU) + 4 * lg) * 8;
                const u4_t lo = *reinterpret_cast<const u4_t*>(p);
                const u4_t hi = *reinterpret_cast<const u4_t*>(p + 16);
                zb[j][0] = __builtin_bit_cast(double, u2_t{lo[0], lo[1]});
                zb[j][1] = __builtin_bit_cast(double, u2_t{lo[2], lo[3]});
                zb[j][2] = __builtin_bit_cast(double, u2_t{hi[0], hi[1]});
                zb[j][3] = __builtin_bit_cast(double, u2_t{hi[2], hi[3]});
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int f = 0; f < WTM; ++f)
#pragma unroll
                    for (int j = 0; j < WTN; ++j)
                        acc[f][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[f][e], zb[j][e], acc[f][j], 0, 0, 0);
        }
    };

    u4_t ra[WTM][2], rn[WTM][2];
    xload(0);
    xstore();
    if (XPRE && a.nb > 1) xload(1);
    aload(ra, 0, 0);
    __syncthreads();
    const int Q = a.Qc + 1;
    for (int64_t i = 0; i < a.nb; ++i) {
        // nU and NG are even, so stages go in pairs and ra ends up holding
        // stage 0 of the next block row
        const int nS = nU + (i > 0 ? NG : 0);
        for (int s = 0; s < nS; s += 2) {
            aload(rn, i, s + 1);
            stage(ra, s);
            if (s + 2 < nS) aload(ra, i, s + 2);
            else if (i + 1 < a.nb) aload(ra, i + 1, 0);
            stage(rn, s + 1);
        }
        // every wave is done with Z_{i-1} and the dosages of block row i
        __syncthreads();
#pragma unroll
        for (int f = 0; f < WTM; ++f)
#pragma unroll
            for (int j = 0; j < WTN; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    *reinterpret_cast<double*>(Zs + (j * 16 + li) * ZS + (rb + f * 16 + lg + 4 * v) * 8) =
                        acc[f][j][v];
        if (i + 1 < a.nb) {
            if (!XPRE) xload(i + 1);
            xstore();
            if (XPRE && i + 2 < a.nb) xload(i + 2);
        }
        // partial sums per 32-row slice (rows i W + rb + 32 h ..)
#pragma unroll
        for (int h = 0; h < WTM / 2; ++h) {
            const int64_t rw = i * W + rb + 32 * h;
            const int64_t pb = rw / 32;
            for (int qq = 0; qq < a.Qc; ++qq) {
                const double* Cq = a.C + qq * a.ldc + rw + lg;
                double cv[2][4];
#pragma unroll
                for (int f = 0; f < 2; ++f)
#pragma unroll
                    for (int v = 0; v < 4; ++v) cv[f][v] = Cq[f * 16 + 4 * v];
#pragma unroll
                for (int j = 0; j < WTN; ++j) {
                    double sum = 0.0;
#pragma unroll
                    for (int f = 0; f < 2; ++f)
#pragma unroll
                        for (int v = 0; v < 4; ++v) sum += acc[2 * h + f][j][v] * cv[f][v];
                    sum = wave_sum16(sum);
                    const int64_t col = c0 + j * 16 + li;
                    if (lg == 0 && col < a.cols) a.part[(pb * Q + qq) * a.ldp + col] = sum;
                }
            }
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
                double sum = 0.0;
#pragma unroll
                for (int f = 0; f < 2; ++f)
#pragma unroll
                    for (int v = 0; v < 4; ++v) sum += acc[2 * h + f][j][v] * acc[2 * h + f][j][v];
                sum = wave_sum16(sum);
                const int64_t col = c0 + j * 16 + li;
                if (lg == 0 && col < a.cols) a.part[(pb * Q + Q - 1) * a.ldp + col] = sum;
            }
        }
#pragma unroll
        for (int f = 0; f < WTM; ++f)
#pragma unroll
            for (int j = 0; j < WTN; ++j) acc[f][j] = d4_t{0.0, 0.0, 0.0, 0.0};
        // Z_i and the next block row's dosages are in place
        __syncthreads();
    }
}

// Block (row0.., col0..) of M, rows x cols, from LAPACK lower band storage
// (M(i, j) at AB[(i - j) + j*ldab] for j <= i <= j + w): entries above the
// diagonal, outside the band or past n are zero, the diagonal past n one.
__global__ void band_block_kernel(const double* __restrict__ AB, int64_t ldab, int64_t w, int64_t n, int64_t row0,
                                  int64_t col0, int64_t rows, int64_t cols, double* __restrict__ out, int64_t ldo) {
    for (int64_t c = blockIdx.x; c < cols; c += gridDim.x)
        for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
            const int64_t i = row0 + r, j = col0 + c;
            double v = 0.0;
            if (i >= j && i - j <= w) {
                if (i < n) v = AB[(i - j) + j * ldab];
                else if (i == j) v = 1.0;
            }
            out[r + c * ldo] = v;
        }
}

}  // namespace

int band_part_rows() { return BT_ROWS; }

hipError_t band_step(const BandArgs& a, hipStream_t s) {
    if (a.cols <= 0) return hipSuccess;
    if (!a.Ut || !a.X || !a.Zcur || !a.part || !a.C || (a.blk > 0 && (!a.Gt || !a.Zprev)))
        return hipErrorInvalidValue;
    if (a.W < BT_M || a.W % 256 || a.blk < 0 || a.n < 1 || a.ldz < a.W || a.ldp < a.cols ||
        a.ldc < (a.blk + 1) * a.W || a.Qc < 1)
        return hipErrorInvalidValue;
    const size_t xs = a.xt == X_I8 ? 1 : 8;
    // 16-byte chunks of a column: the array, its stride and every block's
    // first row (W is a multiple of 256) are 16-byte aligned
    if ((reinterpret_cast<uintptr_t>(a.X) % 16) || ((a.ldx * xs) % 16) ||
        (reinterpret_cast<uintptr_t>(a.Zprev) % 16) || (reinterpret_cast<uintptr_t>(a.Ut) % 16) ||
        (a.Gt && reinterpret_cast<uintptr_t>(a.Gt) % 16))
        return hipErrorInvalidValue;
    if (a.ldx < a.n) return hipErrorInvalidValue;
    const int64_t ctiles = (a.cols + BT_N - 1) / BT_N;
    const int64_t grid = 8 * (a.W / BT_M) * ((ctiles + 7) / 8);
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    // 32-bit buffer offsets: a tile's dosage columns up to the block row's
    // last stage, its rows of U_ii^T and Gt_i^T, its Z columns
    if (((BT_N - 1) * a.ldx + (a.blk + 1) * a.W) * (int64_t)xs > INT32_MAX || (int64_t)BT_M * a.W * 8 > INT32_MAX ||
        (int64_t)BT_N * a.ldz * 8 > INT32_MAX || (reinterpret_cast<uintptr_t>(a.Zcur) % 16))
        return hipErrorInvalidValue;
    if (a.xt == X_I8)
        hipLaunchKernelGGL(band_lds_kernel<int8_t>, dim3((unsigned)grid), dim3(BT_NT), 0, s, a);
    else
        hipLaunchKernelGGL(band_lds_kernel<double>, dim3((unsigned)grid), dim3(BT_NT), 0, s, a);
    return hipGetLastError();
}

// The walk beats one launch per block row (band_lds_kernel) up to W = 512:
// 10.98 against 16.96 ms per 16,384 columns at W = 256 and 20.3 against
// 24.9 at 512 (n = 50,000); from 768 on the launch per block row is faster
// (34.8 against 45.2 ms at 768, 42.1 against 58.1 at 1,024), since 16
// columns per workgroup double the walk's L2 reads per instruction.
bool band_walk_fits(int xt, int64_t W) { return xt == X_I8 && (W == 256 || W == 512); }

hipError_t band_walk(const BandArgs& a, hipStream_t s) {
    if (a.cols <= 0) return hipSuccess;
    if (!band_walk_fits(a.xt, a.W) || a.nb < 1 || !a.Ut || !a.Gt || !a.X || !a.part || !a.C)
        return hipErrorInvalidValue;
    if (a.n < 1 || a.n > a.nb * a.W || a.ldx < a.n || a.ldp < a.cols || a.ldc < a.nb * a.W || a.Qc < 1)
        return hipErrorInvalidValue;
    // 16-byte dosage chunks: the array, its stride and every block's first
    // row are 16-byte aligned; so are the rows of U_ii^T and Gt_i^T
    if ((reinterpret_cast<uintptr_t>(a.X) % 16) || (a.ldx % 16) || (reinterpret_cast<uintptr_t>(a.Ut) % 16) ||
        (reinterpret_cast<uintptr_t>(a.Gt) % 16))
        return hipErrorInvalidValue;
    // columns per workgroup: 32 once a sub-block fills the chip with them,
    // else 16.  W = 256: two workgroups per CU (75 KB of LDS, at most 128
    // VGPRs each); W = 512 keeps 64 rows per wave in more registers, one
    // workgroup per CU.
    const bool wide = a.cols > 8192;
    const int tn = wide ? 32 : 16;
    const int64_t grid = (a.cols + tn - 1) / tn;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    if (a.W == 256) {
        if (wide)
            hipLaunchKernelGGL((band_walk_kernel<2, 2, 4>), dim3((unsigned)grid), dim3(512), 0, s, a);
        else
            hipLaunchKernelGGL((band_walk_kernel<2, 1, 4>), dim3((unsigned)grid), dim3(512), 0, s, a);
    } else {
        if (wide)
            hipLaunchKernelGGL((band_walk_kernel<4, 2, 2>), dim3((unsigned)grid), dim3(512), 0, s, a);
        else
            hipLaunchKernelGGL((band_walk_kernel<4, 1, 2>), dim3((unsigned)grid), dim3(512), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t band_block(const double* AB, int64_t ldab, int64_t w, int64_t n, int64_t row0, int64_t col0, int64_t rows,
                      int64_t cols, double* out, int64_t ldo, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (!AB || !out || ldab < w + 1 || ldo < rows || w < 0) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<int64_t>(cols, 8192);
    hipLaunchKernelGGL(band_block_kernel, dim3(grid), dim3(256), 0, s, AB, ldab, w, n, row0, col0, rows, cols, out,
                       ldo);
    return hipGetLastError();
}

}  // namespace gwas
