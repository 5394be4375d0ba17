// The int8-slice form of the streaming triangular product (Algorithm 2,
// loop body): L^-1 X_blk from int8 digit slices of L^-1 and int8 dosages
// with exact int32 sums on the matrix cores, the slices combined in float64
// in the epilogue, which forms the same partial sums as the floating-point
// product (S_BL, bbar_B and S_BR of Algorithm 2 per wave row slice).
#include "internal.h"
#include "trmm_common.h"

#include <math.h>

#include <algorithm>

namespace gwas {
namespace {

// Accumulator layout of the 16x16x64 int8 instruction: element v of a lane
// holds column lane%16 and row 4*(lane/16) + v.
constexpr int I8_ROW_G = 4, I8_ROW_V = 1;

// Value of the paired digits of one element in units of its row's scale:
// sum_p D_p 2^(-6-7p) / 127^(2p+1), by Horner's rule from the last pair.
// Every shape forms the integers D_p exactly and then this same sequence of
// roundings, so all shapes give the same bits.
template <int NP>
__device__ __forceinline__ double digits_value(const double (&D)[NP]) {
    constexpr double PAIR = 1.0 / (127.0 * 128.0);
    constexpr double UNIT = 1.0 / (127.0 * 64.0);
    double t = D[NP - 1];
#pragma unroll
    for (int p = NP - 2; p >= 0; --p) t = t * PAIR + D[p];
    return t * UNIT;
}

// D_p from one accumulator per digit (exact: |127 acc_hi + acc_lo| < 2^53)
template <int S, int WTN>
__device__ __forceinline__ double digits_of(const i4_t (&acc)[S][WTN], int j, int v) {
    constexpr int NP = (S + 1) / 2;
    double D[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p)
        D[p] = 127.0 * (double)acc[2 * p][j][v] + (2 * p + 1 < S ? (double)acc[2 * p + 1][j][v] : 0.0);
    return digits_value<NP>(D);
}

// L^-1 X from int8 slices of L^-1 and int8 dosages.  Real row r of L^-1 is
// rscale[r] times the value of its paired digits A_s(r, :) (digits_value);
// sliced row R = (r/16)*16*S + s*16 + r%16 holds A_s(r, :) (row-major, K
// contiguous).  Every int32 sum A_s(r, :) x is exact (|sum| <= 64 * 2 * n <
// 2^31), so the float64 combination in the epilogue is the only rounding of
// the product.
// Each wave owns 16 real rows with all S slices (block i = slice i) and
// WTN * 16 SNP columns; the workgroup is WGM x WGN waves.
template <int S, int WGM, int WGN, int WTN, bool GROUPED>
__global__ __launch_bounds__(64 * WGM * WGN) void trmm_sliced_kernel(TrmmArgs la) {
    constexpr int BK = ROW_BYTES;                 // int8 K per stage row
    constexpr int TMR = WGM * 16;                 // real rows per tile
    constexpr int TMS = TMR * S;                  // sliced rows per tile
    constexpr int TN = WGN * WTN * 16;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int A_CHUNKS = TMS * (ROW_BYTES / 16);
    constexpr int CA = (A_CHUNKS + NT - 1) / NT;
    constexpr int B_CHUNKS = TN * (ROW_BYTES / 16);
    constexpr int CB = (B_CHUNKS + NT - 1) / NT;

    const int e0 = la.sched[2 * (int64_t)blockIdx.x];
    const int J = la.sched[2 * (int64_t)blockIdx.x + 1];
    if (e0 < 0) return;
    const int I = e0 & SCHED_ROW_MASK;
    // grouped launches carry one argument set per context; the schedule
    // entry names the context in its high bits.  The set is copied into
    // registers once: read through a reference, every field would be loaded
    // again after each barrier (a barrier is a memory fence).
    const TrmmArgs a = GROUPED ? la.group[__builtin_amdgcn_readfirstlane(e0 >> SCHED_CTX_SHIFT)] : la;
    // a schedule built for more columns than this launch has (sched_cols)
    if ((int64_t)J * TN >= a.cols) return;

    __shared__ __attribute__((aligned(16))) char As[2][TMS * ROW_STRIDE];
    __shared__ __attribute__((aligned(16))) char Bs[2][TN * ROW_STRIDE];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WGN, wc = wave % WGN;
    const int li = lane & 15, lg = lane >> 4;

    const int64_t r0 = (int64_t)I * TMR;                          // first real row
    const int64_t kend = std::min<int64_t>(r0 + TMR, a.n_pad);
    const int64_t nk = (kend + BK - 1) / BK;
    const char* A = reinterpret_cast<const char*>(a.Ut) + (int64_t)I * TMS * a.ldu;
    const int8_t* X = reinterpret_cast<const int8_t*>(a.X);
    const int64_t c0 = (int64_t)J * TN;

    i4_t acc[S][WTN];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = i4_t{0, 0, 0, 0};

    // Staged operands of the next stage: loaded at the top of a stage,
    // written to the other LDS buffer before its barrier.
    u4_t ra[CA], rb[CB];
    auto load = [&](int64_t kt) {
#pragma unroll
        for (int c = 0; c < CA; ++c) {
            const int idx = tid + c * NT;
            if (A_CHUNKS % NT == 0 || idx < A_CHUNKS)
                ra[c] = *reinterpret_cast<const u4_t*>(A + (int64_t)(idx >> 3) * a.ldu + kt * BK + (idx & 7) * 16);
        }
        // whole tile inside the block and the stage inside n: one branch for
        // the workgroup, plain 16-byte loads
        if (c0 + TN <= a.cols && (kt + 1) * BK <= a.n) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int idx = tid + c * NT;
                if (B_CHUNKS % NT == 0 || idx < B_CHUNKS)
                    rb[c] = *reinterpret_cast<const u4_t*>(X + (c0 + (idx >> 3)) * a.ldx + kt * BK + (idx & 7) * 16);
            }
            return;
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int idx = tid + c * NT;
            if (B_CHUNKS % NT == 0 || idx < B_CHUNKS) {
                const int col = idx >> 3, ch = idx & 7;
                const int64_t gcol = c0 + col;
                const int64_t k0 = kt * BK + ch * 16;
                const int8_t* src = X + gcol * a.ldx + k0;
                if (gcol < a.cols && k0 + 16 <= a.n) {
                    rb[c] = *reinterpret_cast<const u4_t*>(src);
                } else {
                    int8_t tmp[16] __attribute__((aligned(16)));
#pragma unroll
                    for (int e = 0; e < 16; ++e) tmp[e] = (gcol < a.cols && k0 + e < a.n) ? src[e] : (int8_t)0;
                    rb[c] = *reinterpret_cast<const u4_t*>(tmp);
                }
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < CA; ++c) {
            const int idx = tid + c * NT;
            if (A_CHUNKS % NT == 0 || idx < A_CHUNKS)
                *reinterpret_cast<u4_t*>(As[buf] + (idx >> 3) * ROW_STRIDE + (idx & 7) * 16) = ra[c];
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int idx = tid + c * NT;
            if (B_CHUNKS % NT == 0 || idx < B_CHUNKS)
                *reinterpret_cast<u4_t*>(Bs[buf] + (idx >> 3) * ROW_STRIDE + (idx & 7) * 16) = rb[c];
        }
    };
    // Fragments of one 64-deep K step (h = 0, 1 of a stage).  (Reading the
    // second step behind the first step's instructions, as the floating-point
    // product does, measured slower here.)
    auto read_step = [&](int buf, int h, u4_t (&fa)[S], u4_t (&fb)[WTN]) {
#pragma unroll
        for (int i = 0; i < S; ++i)
            fa[i] = *reinterpret_cast<const u4_t*>(As[buf] + (wr * S * 16 + i * 16 + li) * ROW_STRIDE + lg * 32 + h * 16);
#pragma unroll
        for (int j = 0; j < WTN; ++j)
            fb[j] = *reinterpret_cast<const u4_t*>(Bs[buf] + (wc * WTN * 16 + j * 16 + li) * ROW_STRIDE + lg * 32 + h * 16);
    };
    auto mma_step = [&](const u4_t (&fa)[S], const u4_t (&fb)[WTN]) {
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(reinterpret_cast<const i4_t&>(fa[i]),
                                                                 reinterpret_cast<const i4_t&>(fb[j]), acc[i][j], 0, 0, 0);
    };
    load(0);
    store(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) load(kt + 1);
        u4_t a0[S], b0[WTN], a1[S], b1[WTN];
        read_step(buf, 0, a0, b0);
        read_step(buf, 1, a1, b1);
        mma_step(a0, b0);
        mma_step(a1, b1);
        // the other buffer held stage kt - 1, which every wave finished
        // reading before the previous barrier
        if (more) store(buf ^ 1);
        __syncthreads();
    }

    // Epilogue: z(r, col) = rscale[r] * the value of the digit sums, then
    // sums over this wave's 16 real rows per column.
    const int Q = a.with_cross ? a.Qc + 1 : 1;
    const int64_t rw = r0 + wr * 16;
    const int64_t pb = rw / 16;
    const int64_t cbase = c0 + wc * WTN * 16 + li;
    double sc[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) sc[v] = a.rscale[rw + I8_ROW_G * lg + I8_ROW_V * v];
    double z[WTN][4];
#pragma unroll
    for (int j = 0; j < WTN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) z[j][v] = sc[v] * digits_of<S, WTN>(acc, j, v);
    if (a.with_cross) {
        for (int q = 0; q < a.Qc; ++q) {
            double cv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) cv[v] = a.C[q * a.ldc + rw + I8_ROW_G * lg + I8_ROW_V * v];
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
                double sum = 0.0;
#pragma unroll
                for (int v = 0; v < 4; ++v) sum += z[j][v] * cv[v];
                sum = wave_sum16(sum);
                const int64_t col = cbase + j * 16;
                if (lg == 0 && col < a.cols) a.part[(pb * Q + q) * a.ldp + col] = sum;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
        double sum = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) sum += z[j][v] * z[j][v];
        sum = wave_sum16(sum);
        const int64_t col = cbase + j * 16;
        if (lg == 0 && col < a.cols) a.part[(pb * Q + Q - 1) * a.ldp + col] = sum;
    }
}

// The same product with its operands loaded straight from global memory
// into LDS (16-byte buffer loads with the LDS destination): no staging
// registers and no LDS write instructions, so a wave's registers go to a
// wider tile.  A stage row is 128 bytes of K with no padding; chunk c of
// row r sits in slot c ^ (r & 7), so the 16 rows a fragment read touches
// fall on distinct banks.  One load instruction of a wave fills 1 KB of
// LDS, 8 rows of 8 slots, lane l writing slot l % 8 of row l / 8.  Reads
// past the dosage block (columns past cols) return zero through the
// buffer range; elements k >= n of a column may hold other data, which
// meets zero entries of L^-1 for every row below n, and rows at or past n
// are zeroed before the epilogue's sums.
template <int S, int WGM, int WGN, int WTN, bool GROUPED>
__global__ __launch_bounds__(64 * WGM * WGN) void trmm_sliced_lds_kernel(TrmmArgs la) {
    constexpr int BK = ROW_BYTES;                 // int8 K per stage row
    constexpr int TMR = WGM * 16;                 // real rows per tile
    constexpr int TMS = TMR * S;                  // sliced rows per tile
    constexpr int TN = WGN * WTN * 16;
    constexpr int NW = WGM * WGN;                 // waves
    constexpr int NA = TMS / 8, NB = TN / 8;      // load instructions (8 rows each) per stage
    static_assert(TMS % 8 == 0 && TN % 8 == 0, "whole load instructions");

    const int e0 = la.sched[2 * (int64_t)blockIdx.x];
    const int J = la.sched[2 * (int64_t)blockIdx.x + 1];
    if (e0 < 0) return;
    const int I = e0 & SCHED_ROW_MASK;
    const TrmmArgs a = GROUPED ? la.group[__builtin_amdgcn_readfirstlane(e0 >> SCHED_CTX_SHIFT)] : la;
    if ((int64_t)J * TN >= a.cols) return;

    __shared__ __attribute__((aligned(1024))) char As[2][TMS * BK];
    __shared__ __attribute__((aligned(1024))) char Bs[2][TN * BK];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WGN, wc = wave % WGN;
    const int li = lane & 15, lg = lane >> 4;

    const int64_t r0 = (int64_t)I * TMR;
    const int64_t kend = std::min<int64_t>(r0 + TMR, a.n_pad);
    const int nk = (int)((kend + BK - 1) / BK);
    const int64_t c0 = (int64_t)J * TN;

    // descriptors: the tile's sliced rows of L^-1; its dosage columns up to
    // the 16-byte chunk holding element n - 1 of the last column in the block
    const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(reinterpret_cast<const char*>(a.Ut) + (int64_t)I * TMS * a.ldu), (short)0,
        (int)(TMS * a.ldu), 0x00020000);
    const int64_t xcols = std::min<int64_t>(TN, a.cols - c0);
    const int64_t xbytes = ((xcols - 1) * a.ldx + a.n + 15) / 16 * 16;
    const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int8_t*>(reinterpret_cast<const int8_t*>(a.X) + c0 * a.ldx), (short)0, (int)xbytes, 0x00020000);
    // this lane's row (column) within each of its load instructions and the
    // swizzled chunk it fetches
    const int lrow = lane >> 3;
    const int lchunk = (lane & 7) ^ (lrow & 7);
    // instruction q of a stage (8 rows) is issued by wave q % NW
    auto load = [&](int kt, int buf) {
#pragma unroll
        for (int c = 0; c < (NA + NW - 1) / NW; ++c) {
            const int q = wave + c * NW;
            if (NA % NW == 0 || q < NA) {
                const int row = q * 8 + lrow;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rsA, (__attribute__((address_space(3))) void*)(As[buf] + q * 8 * BK), 16,
                    (unsigned)(row * a.ldu + kt * BK + lchunk * 16), 0, 0, 0);
            }
        }
#pragma unroll
        for (int c = 0; c < (NB + NW - 1) / NW; ++c) {
            const int q = wave + c * NW;
            if (NB % NW == 0 || q < NB) {
                const int col = q * 8 + lrow;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rsB, (__attribute__((address_space(3))) void*)(Bs[buf] + q * 8 * BK), 16,
                    (unsigned)(col * a.ldx + kt * BK + lchunk * 16), 0, 0, 0);
            }
        }
    };

    i4_t acc[S][WTN];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = i4_t{0, 0, 0, 0};

    // fragment rows start at multiples of 16: row & 7 = li & 7
    const int sw = li & 7;
    auto read_step = [&](int buf, int h, u4_t (&fa)[S], u4_t (&fb)[WTN]) {
        const int slot = ((2 * lg + h) ^ sw) * 16;
#pragma unroll
        for (int i = 0; i < S; ++i)
            fa[i] = *reinterpret_cast<const u4_t*>(As[buf] + (wr * S * 16 + i * 16 + li) * BK + slot);
#pragma unroll
        for (int j = 0; j < WTN; ++j)
            fb[j] = *reinterpret_cast<const u4_t*>(Bs[buf] + (wc * WTN * 16 + j * 16 + li) * BK + slot);
    };
    auto mma_step = [&](const u4_t (&fa)[S], const u4_t (&fb)[WTN]) {
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(reinterpret_cast<const i4_t&>(fa[i]),
                                                                 reinterpret_cast<const i4_t&>(fb[j]), acc[i][j], 0, 0, 0);
    };
    load(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        // the other buffer held stage kt - 1, which every wave finished
        // reading before the previous barrier
        if (kt + 1 < nk) load(kt + 1, buf ^ 1);
        u4_t a0[S], b0[WTN], a1[S], b1[WTN];
        read_step(buf, 0, a0, b0);
        read_step(buf, 1, a1, b1);
        mma_step(a0, b0);
        mma_step(a1, b1);
        // this wave's loads into the other buffer have landed; then every wave's
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }

    const int Q = a.with_cross ? a.Qc + 1 : 1;
    const int64_t rw = r0 + wr * 16;
    const int64_t pb = rw / 16;
    const int64_t cbase = c0 + wc * WTN * 16 + li;
    double sc[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t r = rw + I8_ROW_G * lg + I8_ROW_V * v;
        sc[v] = r < a.n ? a.rscale[r] : 0.0;      // rows past n: zero
    }
    double z[WTN][4];
#pragma unroll
    for (int j = 0; j < WTN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) z[j][v] = sc[v] * digits_of<S, WTN>(acc, j, v);
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
        double sum = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) sum += z[j][v] * z[j][v];
        sum = wave_sum16(sum);
        const int64_t col = cbase + j * 16;
        if (lg == 0 && col < a.cols) a.part[(pb * Q + Q - 1) * a.ldp + col] = sum;
    }
}

// The hi operand of the paired-digit product: bytes x in {0, 1, 2} map to
// 127 (x - 1) in int8 by a byte permute with the dosage bytes as selectors
// into a constant table (the same table in both halves of the permute's
// source pair).
__device__ __forceinline__ uint32_t centred_hi(uint32_t x) {
    return __builtin_amdgcn_perm(0x007f0081u, 0x007f0081u, x);
}

// The product with each pair of digits in one int32 accumulator: the
// instruction for the hi digit A_2p meets 127 (x - 1) and the one for the lo
// digit A_2p+1 meets the dosage bytes themselves, both adding to
// acc_p = sum_k D_p(r, k) x_k - 127 sum_k A_2p(r, k), D_p = 127 A_2p + A_2p+1
// (|127 A_2p (x - 1) + A_2p+1 x| <= 8,256 per k, so |acc_p| < 2^31 for
// n_pad <= 260,096); the epilogue adds the exact row sums
// 127 sum_{k<n} A_2p(r, k) to recover sum_k D_p(r, k) x_k, the same integers
// the other shapes form.  Only the hi operand takes a byte permute.  Half
// the accumulators let a wave hold 16 real rows x WTN * 16 columns with all
// S digits, so each fragment read from LDS feeds more matrix instructions.
// A stage is 64 bytes of K; staged dosage elements past n or past the block
// read as 1 (they meet zero digits).  Dosages must be 0, 1 or 2.
template <int S, int WGM, int WGN, int WTN, bool GROUPED>
__global__ __launch_bounds__(64 * WGM * WGN) void trmm_paired_kernel(TrmmArgs la) {
    constexpr int NP = (S + 1) / 2;
    constexpr int BK = 64;                        // int8 K per stage
    constexpr int RS = BK + 16;                   // LDS row stride (16 rows on distinct banks)
    constexpr int CPR = BK / 16;                  // 16-byte chunks per stage row
    constexpr int TMR = WGM * 16;                 // real rows per tile
    constexpr int TMS = TMR * S;                  // sliced rows per tile
    constexpr int TN = WGN * WTN * 16;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int A_CHUNKS = TMS * CPR;
    constexpr int CA = (A_CHUNKS + NT - 1) / NT;
    constexpr int B_CHUNKS = TN * CPR;
    constexpr int CB = (B_CHUNKS + NT - 1) / NT;

    const int e0 = la.sched[2 * (int64_t)blockIdx.x];
    const int J = la.sched[2 * (int64_t)blockIdx.x + 1];
    if (e0 < 0) return;
    const int I = e0 & SCHED_ROW_MASK;
    const TrmmArgs a = GROUPED ? la.group[__builtin_amdgcn_readfirstlane(e0 >> SCHED_CTX_SHIFT)] : la;
    if ((int64_t)J * TN >= a.cols) return;

    __shared__ __attribute__((aligned(16))) char As[2][TMS * RS];
    __shared__ __attribute__((aligned(16))) char Bs[2][TN * RS];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WGN, wc = wave % WGN;
    const int li = lane & 15, lg = lane >> 4;

    const int64_t r0 = (int64_t)I * TMR;
    const int64_t kend = std::min<int64_t>(r0 + TMR, a.n_pad);
    const int64_t nk = (kend + BK - 1) / BK;
    const char* A = reinterpret_cast<const char*>(a.Ut) + (int64_t)I * TMS * a.ldu;
    const int8_t* X = reinterpret_cast<const int8_t*>(a.X);
    const int64_t c0 = (int64_t)J * TN;

    i4_t acc[NP][WTN];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[p][j] = i4_t{0, 0, 0, 0};

    u4_t ra[CA], rb[CB];
    auto load = [&](int64_t kt) {
#pragma unroll
        for (int c = 0; c < CA; ++c) {
            const int idx = tid + c * NT;
            if (A_CHUNKS % NT == 0 || idx < A_CHUNKS)
                ra[c] = *reinterpret_cast<const u4_t*>(A + (int64_t)(idx / CPR) * a.ldu + kt * BK + (idx % CPR) * 16);
        }
        if (c0 + TN <= a.cols && (kt + 1) * BK <= a.n) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int idx = tid + c * NT;
                if (B_CHUNKS % NT == 0 || idx < B_CHUNKS)
                    rb[c] = *reinterpret_cast<const u4_t*>(X + (c0 + idx / CPR) * a.ldx + kt * BK + (idx % CPR) * 16);
            }
            return;
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int idx = tid + c * NT;
            if (B_CHUNKS % NT == 0 || idx < B_CHUNKS) {
                const int64_t gcol = c0 + idx / CPR;
                const int64_t k0 = kt * BK + (idx % CPR) * 16;
                const int8_t* src = X + gcol * a.ldx + k0;
                if (gcol < a.cols && k0 + 16 <= a.n) {
                    rb[c] = *reinterpret_cast<const u4_t*>(src);
                } else {
                    int8_t tmp[16] __attribute__((aligned(16)));
#pragma unroll
                    for (int e = 0; e < 16; ++e) tmp[e] = (gcol < a.cols && k0 + e < a.n) ? src[e] : (int8_t)1;
                    rb[c] = *reinterpret_cast<const u4_t*>(tmp);
                }
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < CA; ++c) {
            const int idx = tid + c * NT;
            if (A_CHUNKS % NT == 0 || idx < A_CHUNKS)
                *reinterpret_cast<u4_t*>(As[buf] + (idx / CPR) * RS + (idx % CPR) * 16) = ra[c];
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int idx = tid + c * NT;
            if (B_CHUNKS % NT == 0 || idx < B_CHUNKS)
                *reinterpret_cast<u4_t*>(Bs[buf] + (idx / CPR) * RS + (idx % CPR) * 16) = rb[c];
        }
    };

    load(0);
    store(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) load(kt + 1);
        u4_t fa[S], fb[WTN];
#pragma unroll
        for (int i = 0; i < S; ++i)
            fa[i] = *reinterpret_cast<const u4_t*>(As[buf] + (wr * S * 16 + i * 16 + li) * RS + lg * 16);
#pragma unroll
        for (int j = 0; j < WTN; ++j)
            fb[j] = *reinterpret_cast<const u4_t*>(Bs[buf] + (wc * WTN * 16 + j * 16 + li) * RS + lg * 16);
        // hi digits against 127 (x - 1), then lo digits against x: the two
        // instructions into one accumulator are WTN * NP instructions apart
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            u4_t xb[WTN];
#pragma unroll
            for (int j = 0; j < WTN; ++j)
#pragma unroll
                for (int w = 0; w < 4; ++w) xb[j][w] = h == 0 ? centred_hi(fb[j][w]) : fb[j][w];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                if (2 * p + h >= S) continue;
#pragma unroll
                for (int j = 0; j < WTN; ++j)
                    acc[p][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(reinterpret_cast<const i4_t&>(fa[2 * p + h]),
                                                                     reinterpret_cast<const i4_t&>(xb[j]), acc[p][j],
                                                                     0, 0, 0);
            }
        }
        // the other buffer held stage kt - 1, which every wave finished
        // reading before the previous barrier
        if (more) store(buf ^ 1);
        __syncthreads();
    }

    const int Q = a.with_cross ? a.Qc + 1 : 1;
    const int64_t rw = r0 + wr * 16;
    const int64_t pb = rw / 16;
    const int64_t cbase = c0 + wc * WTN * 16 + li;
    double sc[4], rs[NP][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t r = rw + I8_ROW_G * lg + I8_ROW_V * v;
        sc[v] = r < a.n ? a.rscale[r] : 0.0;      // rows past n: zero
#pragma unroll
        for (int p = 0; p < NP; ++p) rs[p][v] = (double)a.rsum[p * a.n_pad + r];
    }
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
        double sum = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double D[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) D[p] = (double)acc[p][j][v] + rs[p][v];
            const double z = sc[v] * digits_value<NP>(D);
            sum += z * z;
        }
        sum = wave_sum16(sum);
        const int64_t col = cbase + j * 16;
        if (lg == 0 && col < a.cols) a.part[(pb * Q + Q - 1) * a.ldp + col] = sum;
    }
}

// Swizzle of the unpadded 64-byte stage rows of the direct-load paired
// shape: chunk c of row r sits in slot c ^ h(r % 16).  A fragment read
// touches rows base + 0..15 (base a multiple of 16) at one chunk; h sends
// the rows that share banks to distinct slots, whether the LDS serves 8 or
// 16 lanes of a 16-byte read per cycle.
__device__ __forceinline__ int pair_swz(int r) { return ((r >> 2) & 1) | ((((r >> 1) ^ (r >> 3)) & 1) << 1); }
// The same for 128-byte stage rows (8 chunks): chunk c of row r in slot
// c ^ ((r % 8) ^ bit 3 of r).
__device__ __forceinline__ int pair_swz8(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// The paired-digit product with its operands loaded straight from global
// memory into NBUF LDS buffers (2 or 3): the loads of stage kt + NBUF - 1
// are issued at the top of stage kt, and with three buffers the end of
// stage kt waits only for stage kt + 1's loads, so two stages of matrix
// instructions cover their latency (the stage barrier is a bare s_barrier:
// a memory fence there would wait for every load in flight).  A stage is
// BK = 64 or 128 bytes of K (one or two instruction steps per barrier).
// Shapes of four waves run two workgroups per CU, whose barriers fall at
// different times.  Reads past the dosage block return zero
// through the buffer range; elements k >= n of a column may hold other
// data, which meets zero digits of every row below n, and rows at or past
// n get a zero scale.
template <int S, int WGM, int WGN, int WTN, int NBUF, int BK, bool GROUPED>
__global__ __launch_bounds__(64 * WGM * WGN, 2) void trmm_paired_lds_kernel(TrmmArgs la) {
    static_assert(NBUF == 2 || NBUF == 3, "two or three stage buffers");
    static_assert(BK == 64 || BK == 128, "stage rows of 64 or 128 bytes of K");
    constexpr int LOOK = NBUF - 1;                // stages loaded ahead
    constexpr int NP = (S + 1) / 2;
    constexpr int CPR = BK / 16;                  // 16-byte chunks per stage row
    constexpr int RPI = 1024 / BK;                // rows per load instruction (1 KB)
    constexpr int TMR = WGM * 16;
    constexpr int TMS = TMR * S;
    constexpr int TN = WGN * WTN * 16;
    constexpr int NW = WGM * WGN;
    constexpr int NA = TMS / RPI, NB = TN / RPI;  // load instructions per stage
    static_assert(NB % NW == 0, "every wave issues the same number of dosage loads");
    // instruction q is issued by wave q % NW: the first NA % NW waves issue
    // one more L^-1 load per stage than the others
    constexpr int LA = (NA + NW - 1) / NW, LB = NB / NW;
    static_assert(LA + LB < 16, "vmcnt field");
    // s_waitcnt immediates: vmcnt(this wave's loads per stage) or vmcnt(0),
    // with lgkmcnt(0) and any expcnt
    constexpr int WAIT_MORE = (LA + LB) | (7 << 4);
    constexpr int WAIT_LESS = (NA % NW == 0 ? LA + LB : LA - 1 + LB) | (7 << 4);
    constexpr int WAIT_ALL = 7 << 4;

    const int e0 = la.sched[2 * (int64_t)blockIdx.x];
    const int J = la.sched[2 * (int64_t)blockIdx.x + 1];
    if (e0 < 0) return;
    const int I = e0 & SCHED_ROW_MASK;
    const TrmmArgs a = GROUPED ? la.group[__builtin_amdgcn_readfirstlane(e0 >> SCHED_CTX_SHIFT)] : la;
    if ((int64_t)J * TN >= a.cols) return;

    __shared__ __attribute__((aligned(1024))) char Abuf[NBUF][TMS * BK];
    __shared__ __attribute__((aligned(1024))) char Bbuf[NBUF][TN * BK];
    char* const A0 = Abuf[0];
    char* const A1 = Abuf[1];
    char* const A2 = Abuf[NBUF - 1];
    char* const B0 = Bbuf[0];
    char* const B1 = Bbuf[1];
    char* const B2 = Bbuf[NBUF - 1];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WGN, wc = wave % WGN;
    const int li = lane & 15, lg = lane >> 4;

    const int64_t r0 = (int64_t)I * TMR;
    const int64_t kend = std::min<int64_t>(r0 + TMR, a.n_pad);
    const int nk = (int)((kend + BK - 1) / BK);
    const int64_t c0 = (int64_t)J * TN;

    const u4_t rsA = buffer_words(reinterpret_cast<const char*>(a.Ut) + (int64_t)I * TMS * a.ldu,
                                  (uint32_t)(TMS * a.ldu));
    const int64_t xcols = std::min<int64_t>(TN, a.cols - c0);
    const int64_t xbytes = ((xcols - 1) * a.ldx + a.n + 15) / 16 * 16;
    const u4_t rsB = buffer_words(reinterpret_cast<const int8_t*>(a.X) + c0 * a.ldx, (uint32_t)xbytes);
    // lane l of a load instruction fills slot l % CPR of row l / CPR of its
    // RPI rows with the chunk that belongs there (for 128-byte rows the
    // swizzle of the row depends on the parity of the instruction's group)
    const int lrow = lane / CPR;
    auto lchunk = [&](int q) {
        return BK == 64 ? (lane & 3) ^ pair_swz(lrow) : (lane & 7) ^ pair_swz8(q * RPI + lrow);
    };
    // instruction q of a stage (RPI rows) is issued by wave q % NW
    auto load = [&](int kt, char* Ab, char* Bb) {
#pragma unroll
        for (int c = 0; c < LA; ++c) {
            const int q = wave + c * NW;
            if (NA % NW != 0 && q >= NA) break;
            load_lds16(rsA, lds_address(Ab + q * 1024),
                       (uint32_t)((q * RPI + lrow) * a.ldu + kt * BK + lchunk(q) * 16));
        }
#pragma unroll
        for (int c = 0; c < LB; ++c) {
            const int q = wave + c * NW;
            load_lds16(rsB, lds_address(Bb + q * 1024),
                       (uint32_t)((q * RPI + lrow) * a.ldx + kt * BK + lchunk(q) * 16));
        }
    };

    i4_t acc[NP][WTN];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[p][j] = i4_t{0, 0, 0, 0};

    const bool more_a = NA % NW == 0 || wave < NA % NW;   // wave-uniform
    auto stage = [&](int kt, const char* Ar, const char* Br, char* An, char* Bn) {
        const bool ahead = kt + LOOK < nk;
        if (ahead) load(kt + LOOK, An, Bn);
#pragma unroll
        for (int ks = 0; ks < BK / 64; ++ks) {
            // chunk 4 ks + lg of the fragment's rows (row bases are multiples of 16)
            const int slot = (BK == 64 ? lg ^ pair_swz(li) : (4 * ks + lg) ^ pair_swz8(li)) * 16;
            u4_t fa[S], fb[WTN];
#pragma unroll
            for (int i = 0; i < S; ++i)
                fa[i] = *reinterpret_cast<const u4_t*>(Ar + (wr * S * 16 + i * 16 + li) * BK + slot);
#pragma unroll
            for (int j = 0; j < WTN; ++j)
                fb[j] = *reinterpret_cast<const u4_t*>(Br + (wc * WTN * 16 + j * 16 + li) * BK + slot);
            // hi digits against 127 (x - 1), then lo digits against x, one
            // dosage fragment at a time (its byte map just before its
            // instructions); the two instructions into one accumulator are
            // WTN * NP instructions apart
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int j = 0; j < WTN; ++j) {
                    u4_t xb;
#pragma unroll
                    for (int w = 0; w < 4; ++w) xb[w] = h == 0 ? centred_hi(fb[j][w]) : fb[j][w];
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        if (2 * p + h >= S) continue;
                        acc[p][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            reinterpret_cast<const i4_t&>(fa[2 * p + h]), reinterpret_cast<const i4_t&>(xb), acc[p][j],
                            0, 0, 0);
                    }
                }
        }
        // the stage's matrix instructions stay ahead of its barrier (the
        // compiler would sink them below it, and the wait for the next
        // stage's loads would no longer overlap them)
        __builtin_amdgcn_sched_barrier(0);
        // stage kt + 1 has landed (this wave's part), and this wave's reads
        // of stage kt are done before any wave may load into its buffer
        if (LOOK == 1 || !ahead) __builtin_amdgcn_s_waitcnt(WAIT_ALL);
        else if (more_a) __builtin_amdgcn_s_waitcnt(WAIT_MORE);
        else __builtin_amdgcn_s_waitcnt(WAIT_LESS);
        compiler_fence();
        __builtin_amdgcn_s_barrier();
        compiler_fence();
    };

    load(0, A0, B0);
    if (LOOK == 2 && nk > 1) {
        load(1, A1, B1);
        if (more_a) __builtin_amdgcn_s_waitcnt(WAIT_MORE);
        else __builtin_amdgcn_s_waitcnt(WAIT_LESS);
    } else {
        __builtin_amdgcn_s_waitcnt(WAIT_ALL);
    }
    compiler_fence();
    __builtin_amdgcn_s_barrier();
    compiler_fence();
    if constexpr (NBUF == 3) {
        for (int kt = 0; kt < nk; kt += 3) {
            stage(kt, A0, B0, A2, B2);
            if (kt + 1 < nk) stage(kt + 1, A1, B1, A0, B0);
            if (kt + 2 < nk) stage(kt + 2, A2, B2, A1, B1);
        }
    } else {
        for (int kt = 0; kt < nk; kt += 2) {
            stage(kt, A0, B0, A1, B1);
            if (kt + 1 < nk) stage(kt + 1, A1, B1, A0, B0);
        }
    }

    const int Q = a.with_cross ? a.Qc + 1 : 1;
    const int64_t rw = r0 + wr * 16;
    const int64_t pb = rw / 16;
    const int64_t cbase = c0 + wc * WTN * 16 + li;
    double sc[4], rs[NP][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t r = rw + I8_ROW_G * lg + I8_ROW_V * v;
        sc[v] = r < a.n ? a.rscale[r] : 0.0;      // rows past n: zero
#pragma unroll
        for (int p = 0; p < NP; ++p) rs[p][v] = (double)a.rsum[p * a.n_pad + r];
    }
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
        double sum = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double D[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) D[p] = (double)acc[p][j][v] + rs[p][v];
            const double z = sc[v] * digits_value<NP>(D);
            sum += z * z;
        }
        sum = wave_sum16(sum);
        const int64_t col = cbase + j * 16;
        if (lg == 0 && col < a.cols) a.part[(pb * Q + Q - 1) * a.ldp + col] = sum;
    }
}

}  // namespace

// Shapes of the int8-slice product: 0, operands staged through registers
// (32 real rows x 256 columns); 1, the same tile loaded straight into LDS;
// 2, loaded straight into LDS with waves of 16 x 80 (32 x 320); paired
// digits: 3, waves of 16 x 128 staged through registers (64 x 256); 4, the
// same tile loaded straight into three LDS buffers; 5, 4 waves of 16 x 128
// (32 x 256), two LDS buffers, two workgroups per CU; 6, as 4 with 128-byte
// stages in two LDS buffers (all 160 KB of a CU's LDS).
int trmm_sliced_cfgs() { return 7; }
TrmmShape trmm_sliced_shape(int cfg) {
    switch (cfg) {
        case 2: return TrmmShape{2 * 16, 4 * 5 * 16, 16, 512, 1, 32};
        case 3: case 4: case 6: return TrmmShape{4 * 16, 2 * 8 * 16, 16, 512, 1, 32};
        case 5: return TrmmShape{2 * 16, 2 * 8 * 16, 16, 256, 1, 32};
        default: return TrmmShape{2 * 16, 4 * 4 * 16, 16, 512, 1, 32};
    }
}
bool trmm_sliced_two_per_cu(int cfg) { return cfg == 5; }
// The paired-digit 64 x 256 tile with 128-byte stages in two LDS buffers,
// one workgroup per CU: 0.509 of int8 peak at n = 50k and 100k, against
// 0.493 and 0.496 with 64-byte stages in three buffers (shape 4); the
// two-workgroup 32 x 256 shape is a little faster at 50k (0.50) but falls to
// 0.33 from 75k on, and the unpaired register-staged tile gives 0.42-0.44.
int trmm_sliced_default_cfg() { return 6; }
bool trmm_sliced_paired(int cfg) { return cfg >= 3; }
bool trmm_sliced_direct(int cfg) { return cfg == 1 || cfg == 2 || cfg >= 4; }

namespace {
template <bool G>
hipError_t launch_sliced(const TrmmArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)a.n_sched), block(512), block4(256);
#define GWAS_SLICED_CASE(S)                                                                            \
    case S:                                                                                            \
        if (a.cfg == 0) hipLaunchKernelGGL((trmm_sliced_kernel<S, 2, 4, 4, G>), grid, block, 0, s, a);       \
        else if (a.cfg == 1) hipLaunchKernelGGL((trmm_sliced_lds_kernel<S, 2, 4, 4, G>), grid, block, 0, s, a); \
        else if (a.cfg == 2) hipLaunchKernelGGL((trmm_sliced_lds_kernel<S, 2, 4, 5, G>), grid, block, 0, s, a); \
        else if (a.cfg == 3) hipLaunchKernelGGL((trmm_paired_kernel<S, 4, 2, 8, G>), grid, block, 0, s, a);    \
        else if (a.cfg == 4) hipLaunchKernelGGL((trmm_paired_lds_kernel<S, 4, 2, 8, 3, 64, G>), grid, block, 0, s, a); \
        else if (a.cfg == 5) hipLaunchKernelGGL((trmm_paired_lds_kernel<S, 2, 2, 8, 2, 64, G>), grid, block4, 0, s, a); \
        else if (a.cfg == 6) hipLaunchKernelGGL((trmm_paired_lds_kernel<S, 4, 2, 8, 2, 128, G>), grid, block, 0, s, a); \
        else return hipErrorInvalidValue;                                                               \
        return hipGetLastError();
    switch (a.slices) {
        GWAS_SLICED_CASE(4) GWAS_SLICED_CASE(5) GWAS_SLICED_CASE(6)
        default: return hipErrorInvalidValue;
    }
#undef GWAS_SLICED_CASE
}
}  // namespace

// Arguments were checked by trmm_check (single launches) or by the caller
// (grouped launches).
hipError_t trmm_sliced_launch(const TrmmArgs& a, hipStream_t s) {
    return a.group ? launch_sliced<true>(a, s) : launch_sliced<false>(a, s);
}

}  // namespace gwas
