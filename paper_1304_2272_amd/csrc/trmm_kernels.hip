// The streaming triangular product of the per-block hot path (Algorithm 2,
// loop body): Xbar_blk = L^-1 X_blk on matrix cores, never stored, with the
// cross products of Algorithm 2 fused into its epilogue (S_BL = xbar^T
// Xbar_L, bbar_B = xbar^T ybar, S_BR = xbar^T xbar) as partial sums per
// wave row slice; tile shapes, their XCD schedule, argument checks and the
// launcher (the int8-slice form of the product has its own source).
#include "internal.h"
#include "trmm_common.h"

#include <math.h>
#include <stdlib.h>

#include <algorithm>
#include <type_traits>
#include <vector>

namespace gwas {
namespace {

// Reduced-precision sums move to float64 every FLUSH_STAGES stages in the
// shapes that keep float64 sums.  At n = 50,000 the float32 error of b
// against the float64 path is 5.5e-11 flushing every 4 stages, 6.3e-11
// every 16 and 2.0e-10 to 4e-10 with float32 sums only: rounding L^-1 to
// float32 dominates.  16 stages saves 2% of the float32 product's time
// over 4.
constexpr int FLUSH_STAGES = 16;

// Accumulator layout of the 16x16 instructions: element v of a lane holds
// column lane%16 and row ROW_G*(lane/16) + ROW_V*v.  NQ: sub-steps a lane's
// 32-byte K slice of a stage is read in (see trmm_stream_kernel).
template <typename AT> struct MM;
template <> struct MM<double> {
    static constexpr int BK = 16, KPL = 1, NQ = 4;
    static constexpr int ROW_G = 1, ROW_V = 4;
    typedef d4_t acc_t;
    typedef double frag_t;
    __device__ static acc_t mma(frag_t a, frag_t b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct MM<float> {
    static constexpr int BK = 32, KPL = 1, NQ = 4;
    static constexpr int ROW_G = 4, ROW_V = 1;
    typedef f4_t acc_t;
    typedef float frag_t;
    __device__ static acc_t mma(frag_t a, frag_t b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct MM<__bf16> {
    static constexpr int BK = 64, KPL = 8, NQ = 2;
    static constexpr int ROW_G = 4, ROW_V = 1;
    typedef f4_t acc_t;
    typedef bf8_t frag_t;
    __device__ static acc_t mma(frag_t a, frag_t b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

template <typename AT> __device__ __forceinline__ AT from_i8(int8_t x) { return (AT)(int)x; }
template <typename AT> __device__ __forceinline__ AT from_f64(double x) { return (AT)x; }
template <> __device__ __forceinline__ __bf16 from_f64<__bf16>(double x) { return (__bf16)(float)x; }

// Operand of instruction s from a lane's 8- or 16-byte fragment piece.  A
// vector element is copied to a scalar before its bit cast: hipcc's
// __builtin_bit_cast of an element expression v[s] reads element 0.
template <typename AT>
__device__ __forceinline__ typename MM<AT>::frag_t frag(const u4_t& f, int s) {
    if constexpr (sizeof(AT) == 8) {
        return __builtin_bit_cast(double, u2_t{f[2 * s], f[2 * s + 1]});
    } else if constexpr (sizeof(AT) == 4) {
        const uint32_t w = f[s];
        return __builtin_bit_cast(float, w);
    } else {
        return __builtin_bit_cast(bf8_t, f);
    }
}
template <typename AT>
__device__ __forceinline__ typename MM<AT>::frag_t frag(const u2_t& f, int s) {
    if constexpr (sizeof(AT) == 8) {
        return __builtin_bit_cast(double, f);
    } else {
        static_assert(sizeof(AT) == 4, "8-byte pieces hold float64 or float32 operands");
        const uint32_t w = f[s];
        return __builtin_bit_cast(float, w);
    }
}
template <int BYTES> struct Piece { typedef u4_t type; };
template <> struct Piece<8> { typedef u2_t type; };

// Workgroup shape: WGM x WGN waves, each wave WTM x WTN blocks of 16 x 16.
// SUM32: the reduced-precision products keep float32 sums only, with no
// float64 sums beside them (whose registers limit a wave to 64 x 64).
template <int WGM_, int WGN_, int WTM_, int WTN_, int MINB_, bool SUM32_ = false> struct Shape {
    static constexpr int WGM = WGM_, WGN = WGN_, WTM = WTM_, WTN = WTN_, MINB = MINB_;
    static constexpr bool SUM32 = SUM32_;
    static constexpr int TM = WGM * WTM * 16;     // rows of L^-1 / Z per tile
    static constexpr int TN = WGN * WTN * 16;     // SNP columns per tile
    static constexpr int NT = 64 * WGM * WGN;     // threads
};

// Segments of the bfloat16-slice product: the K range runs once per pair
// (slice i of L^-1, slice j of the dosages) with i + j <= 2, smallest
// first, all into the same sums.  Three slices of L^-1 with int8 dosages
// (exact in bfloat16): (2,0), (1,0), (0,0); with float64 dosages, cut into
// three slices as well (once per sub-block, before the product):
// (2,0), (1,1), (0,2), (1,0), (0,1), (0,0).
__device__ __forceinline__ int seg_a(int nseg, int s) {
    if (nseg == 3) return 2 - s;
    if (nseg == 6) return s == 0 ? 2 : (s == 1 || s == 3) ? 1 : 0;
    return 0;
}
__device__ __forceinline__ int seg_x(int nseg, int s) {
    if (nseg == 6) return (s == 1 || s == 4) ? 1 : s == 2 ? 2 : 0;
    return 0;
}

// One TM x TN tile of Z = L^-1 X per workgroup.  The tile's K range is
// [0, r0 + TM) because L^-1 is lower triangular.  Stages of 128 bytes of K
// per row go global -> registers -> LDS (double buffered); within a stage
// lane group g = lane/16 supplies the contiguous K slice [g*BK/4, (g+1)*BK/4)
// to A and B alike.  Tile coordinates come from the schedule.
template <typename AT, typename XT, typename S, bool GROUPED>
__global__ __launch_bounds__(S::NT, S::MINB) void trmm_stream_kernel(TrmmArgs la) {
    typedef MM<AT> T;
    constexpr int BK = T::BK;
    constexpr bool LOWP = sizeof(AT) < 8;
    // dosages given as three bfloat16 slices (the bfloat16-slice product
    // with float64 dosages): segment s reads slice seg_x(s)
    constexpr bool XSL = std::is_same<XT, __bf16>::value;
    // reduced-precision sums move to float64 registers every FLUSH_STAGES
    // stages unless the shape keeps float32 sums only
    constexpr bool SUM64 = LOWP && !S::SUM32;
    constexpr int TM = S::TM, TN = S::TN, NT = S::NT, WTM = S::WTM, WTN = S::WTN;
    constexpr int A_CHUNKS = TM * (ROW_BYTES / 16);              // 16-byte chunks per stage
    constexpr int CA = (A_CHUNKS + NT - 1) / NT;
    constexpr int XB = BK * (int)sizeof(XT);                     // bytes of one column per stage
    constexpr int CPC = XB / 16;                                 // 16-byte chunks per column
    constexpr int EPC = 16 / (int)sizeof(XT);                    // elements per chunk
    constexpr int B_CHUNKS = TN * CPC;
    constexpr int CB = (B_CHUNKS + NT - 1) / NT;
    static_assert(XB % 16 == 0, "a column stage must be whole 16-byte chunks");

    // the tile coordinates are the workgroup's: scalar registers, so that
    // every quantity derived from them (K range, addresses, loop bound) is
    // scalar too
    const int e0 = __builtin_amdgcn_readfirstlane(la.sched[2 * (int64_t)blockIdx.x]);
    const int J = __builtin_amdgcn_readfirstlane(la.sched[2 * (int64_t)blockIdx.x + 1]);
    if (e0 < 0) return;
    const int I = e0 & SCHED_ROW_MASK;
    // grouped launches carry one argument set per context; the schedule
    // entry names the context in its high bits.  The set is copied into
    // registers once: read through a reference, every field would be loaded
    // again after each barrier (a barrier is a memory fence).
    const TrmmArgs a = GROUPED ? la.group[e0 >> SCHED_CTX_SHIFT] : la;
    // a schedule built for more columns than this launch has (sched_cols)
    if ((int64_t)J * TN >= a.cols) return;

    __shared__ __attribute__((aligned(16))) char As[2][TM * ROW_STRIDE];
    __shared__ __attribute__((aligned(16))) char Bs[2][TN * ROW_STRIDE];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave / S::WGN, wc = wave % S::WGN;
    const int li = lane & 15, lg = lane >> 4;

    const int64_t r0 = (int64_t)I * TM;
    const int64_t c0 = (int64_t)J * TN;
    // L^-1 is lower triangular: its rows r0.. end at column r0 + TM; a full
    // matrix (M^-1 in the reverse pass) runs the whole K range
    const int64_t kend = a.full_k ? a.n_pad : std::min<int64_t>(r0 + TM, a.n_pad);
    // stage index: 32-bit where registers are short (SUM32 shapes)
    typedef typename std::conditional<S::SUM32, int, int64_t>::type kidx_t;
    const kidx_t nk = (kidx_t)(kend / BK);
    // the bfloat16-slice product (a.slices == 3) runs the K range once per
    // segment; slice i of L^-1 starts i * n_pad elements into each row
    const int nseg = (sizeof(AT) == 2 && a.slices == 3) ? (sizeof(XT) == 1 ? 3 : 6) : 1;
    const kidx_t nkt = nk * (kidx_t)nseg;
    const int64_t seg_bytes = a.n_pad * (int64_t)sizeof(AT);
    int xj_next = 0;   // dosage slice of the segment being loaded (bfloat16 slices)
    const char* Ut = reinterpret_cast<const char*>(a.Ut);
    const int64_t row_bytes = a.ldu * (int64_t)sizeof(AT);
    const XT* X = reinterpret_cast<const XT*>(a.X);

    typename T::acc_t acc[WTM][WTN];
    d4_t acc64[SUM64 ? WTM : 1][SUM64 ? WTN : 1];
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = typename T::acc_t{0, 0, 0, 0};
    if constexpr (SUM64) {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j) acc64[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
    }

    u4_t ra[CA], rb[CB];
    // Buffer loads (SUM32 shapes, whose registers are short): 32-bit
    // offsets from a per-tile base.  L^-1 takes its chunk and stage offsets
    // in scalar registers and never leaves the tile's rows.  The dosage
    // offset is all in the vector operand, which the descriptor's range
    // check covers: chunks past the block's data read as zero (chunks are
    // 16-byte aligned in every column, since ldx bytes are a multiple of
    // 16), and elements k >= n of the last stages are cleared here.
    constexpr bool BUF = S::SUM32;
    __amdgpu_buffer_rsrc_t rsA, rsB;
    int voA = 0, voB = 0;
    if constexpr (BUF) {
        static_assert(A_CHUNKS % NT == 0 && B_CHUNKS % NT == 0 && NT % CPC == 0, "whole chunks per lane");
        rsA = __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(Ut + r0 * row_bytes), (short)0,
                                                (int)(TM * row_bytes), 0x00020000);
        // the range ends with the 16-byte chunk that holds element n - 1 of
        // the tile's last column: the caller's array need not extend to ldx
        // there
        const int64_t xcols = std::min<int64_t>(TN, a.cols - c0);
        // bfloat16 slices of float64 dosages: the last column's third slice
        const int64_t xbytes = ((xcols - 1) * a.ldx + (XSL && nseg > 1 ? 2 * a.n_pad : 0) + a.n) * (int64_t)sizeof(XT);
        rsB = __builtin_amdgcn_make_buffer_rsrc(const_cast<XT*>(X + c0 * a.ldx), (short)0,
                                                (int)((xbytes + 15) / 16 * 16), 0x00020000);
        voA = (tid >> 3) * (int)row_bytes + (tid & 7) * 16;
        voB = (tid / CPC) * (int)(a.ldx * (int64_t)sizeof(XT)) + (tid % CPC) * 16;
    }
    auto load_buf = [&](int kt) {
        int ai = 0;
        int xo = 0;   // bytes to the dosage slice of the segment (bfloat16 slices)
        if (nseg > 1) {
            const int seg = kt / (int)nk;
            kt -= seg * (int)nk;
            ai = seg_a(nseg, seg);
            xj_next = seg_x(nseg, seg);
            if constexpr (XSL) xo = xj_next * (int)(a.n_pad * (int64_t)sizeof(XT));
        }
#pragma unroll
        for (int c = 0; c < CA; ++c)
            ra[c] = __builtin_bit_cast(u4_t, __builtin_amdgcn_raw_buffer_load_b128(
                                                 rsA, voA, (int)(c * (NT / 8) * row_bytes + kt * ROW_BYTES + ai * seg_bytes), 0));
#pragma unroll
        for (int c = 0; c < CB; ++c)
            rb[c] = __builtin_bit_cast(u4_t, __builtin_amdgcn_raw_buffer_load_b128(
                                                 rsB, voB + (int)(c * (NT / CPC) * a.ldx * (int64_t)sizeof(XT)) + kt * XB + xo, 0, 0));
        if ((kt + 1) * BK > (int)a.n) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                // bytes of this chunk below n
                const int k0 = kt * BK + ((tid + c * NT) % CPC) * EPC;
                const int vb = std::min(16, std::max(0, ((int)a.n - k0) * (int)sizeof(XT)));
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int keep = std::min(4, std::max(0, vb - 4 * w));
                    rb[c][w] &= keep >= 4 ? 0xffffffffu : ((1u << (8 * keep)) - 1u);
                }
            }
        }
    };
    auto load = [&](kidx_t kt) {
        if constexpr (BUF) {
            load_buf(kt);
            return;
        }
        int64_t aoff = 0;
        const XT* Xs = X;   // the segment's dosage slice (bfloat16 slices)
        if (nseg > 1) {
            const kidx_t seg = kt / nk;
            kt -= seg * nk;
            aoff = seg_a(nseg, (int)seg) * seg_bytes;
            xj_next = seg_x(nseg, (int)seg);
            if constexpr (XSL) Xs = X + xj_next * a.n_pad;
        }
#pragma unroll
        for (int c = 0; c < CA; ++c) {
            const int idx = tid + c * NT;
            if (A_CHUNKS % NT == 0 || idx < A_CHUNKS) {
                const int row = idx >> 3, ch = idx & 7;
                ra[c] = *reinterpret_cast<const u4_t*>(Ut + (r0 + row) * row_bytes + aoff + kt * ROW_BYTES + ch * 16);
            }
        }
        // Whole tile inside the block and the stage inside n: one branch for
        // the workgroup and plain 16-byte loads.  This pays where a stage
        // holds few matrix-core cycles (float32, bfloat16); the float64
        // product measured faster with the per-lane checks alone.
        if constexpr (sizeof(AT) < 8) {
            if (c0 + TN <= a.cols && (kt + 1) * BK <= a.n) {
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    const int idx = tid + c * NT;
                    if (B_CHUNKS % NT == 0 || idx < B_CHUNKS) {
                        const int col = idx / CPC, ch = idx % CPC;
                        rb[c] = *reinterpret_cast<const u4_t*>(Xs + (c0 + col) * a.ldx + kt * BK + ch * EPC);
                    }
                }
                return;
            }
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int idx = tid + c * NT;
            if (B_CHUNKS % NT == 0 || idx < B_CHUNKS) {
                const int col = idx / CPC, ch = idx % CPC;
                const int64_t gcol = c0 + col;
                const int64_t k0 = kt * BK + ch * EPC;
                const XT* src = Xs + gcol * a.ldx + k0;
                if constexpr (sizeof(AT) == 8) {
                    // A chunk whose column is in the block and whose first
                    // element is below n lies inside the caller's array (ldx
                    // bytes are a multiple of 16): load it whole and clear its
                    // elements k >= n in registers, so the chunk stays one
                    // 16-byte value on every path and the compiler need not
                    // unpack it (and wait for it) right after the load.
                    u4_t v = u4_t{0u, 0u, 0u, 0u};
                    if (gcol < a.cols && k0 < a.n) v = *reinterpret_cast<const u4_t*>(src);
                    if (k0 + EPC > a.n) {
                        const int vb = (int)std::min<int64_t>(16, std::max<int64_t>(0, (a.n - k0) * (int64_t)sizeof(XT)));
#pragma unroll
                        for (int w = 0; w < 4; ++w) {
                            const int keep = std::min(4, std::max(0, vb - 4 * w));
                            v[w] &= keep >= 4 ? 0xffffffffu : ((1u << (8 * keep)) - 1u);
                        }
                    }
                    rb[c] = v;
                } else if (gcol < a.cols && k0 + EPC <= a.n) {
                    rb[c] = *reinterpret_cast<const u4_t*>(src);
                } else {
                    XT tmp[EPC] __attribute__((aligned(16)));
#pragma unroll
                    for (int e = 0; e < EPC; ++e) tmp[e] = (gcol < a.cols && k0 + e < a.n) ? src[e] : (XT)0;
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
            // An empty register-only asm: the float64 product's dosage chunk
            // is taken apart here, not right after its load, where the
            // compiler would otherwise move the unpacking and wait for the
            // load (+2%; the reduced-precision shapes measured slower or
            // spilled with it).
            if constexpr (sizeof(AT) == 8) asm volatile("" : "+v"(rb[c]));
            const int idx = tid + c * NT;
            if (B_CHUNKS % NT == 0 || idx < B_CHUNKS) {
                const int col = idx / CPC, ch = idx % CPC;
                AT* dst = reinterpret_cast<AT*>(Bs[buf] + col * ROW_STRIDE) + ch * EPC;
                if constexpr (XSL) {
                    // dosages cut to bfloat16 go in as they are
                    *reinterpret_cast<u4_t*>(dst) = rb[c];
                } else {
                    const XT* x = reinterpret_cast<const XT*>(&rb[c]);
#pragma unroll
                    for (int e = 0; e < EPC; ++e) {
                        if constexpr (sizeof(XT) == 1) dst[e] = from_i8<AT>((int8_t)x[e]);
                        else dst[e] = from_f64<AT>((double)x[e]);
                    }
                }
            }
        }
    };

    auto flush = [&]() {
        if constexpr (SUM64) {
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int j = 0; j < WTN; ++j) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc64[i][j][v] += (double)acc[i][j][v];
                    acc[i][j] = typename T::acc_t{0, 0, 0, 0};
                }
        }
    };
    // the product's value at accumulator (i, j, v), in float64
    auto zval = [&](int i, int j, int v) -> double {
        if constexpr (SUM64) return acc64[i][j][v];
        else return (double)acc[i][j][v];
    };
    // A lane's K slice of a stage (32 bytes of A and of B per 16-row block)
    // is read in NQ pieces into two alternating register sets: piece q + 1
    // is read while piece q's matrix instructions run, and the next stage's
    // first piece is read right after the barrier, behind the last piece's
    // instructions, so no wave waits on LDS at a stage boundary.  NQ = 1
    // reads the whole slice before the stage's instructions (for tiles with
    // no registers to spare).
    // 64 x 64 waves of the reduced-precision products carry float64 sums
    // besides their float32 ones; two of them per SIMD leave no registers
    // for a second set.
    // 64 x 128 waves (SUM32) keep the pieces of a stage inside it (a set
    // carried over the barrier spills): float32 in 8-byte pieces with two
    // sets, bfloat16 (whose instruction takes 16 bytes) in 16-byte pieces
    // with one set.
    constexpr bool TIGHT = (NT / 64) * S::MINB > 4;
    constexpr int NQ = S::SUM32 ? (sizeof(AT) == 4 ? 4 : 2)
                                : ((SUM64 && TIGHT && WTM * WTN >= 16) ? 1 : T::NQ);
    constexpr int SETS = (S::SUM32 && sizeof(AT) != 4) ? 1 : 2;
    constexpr int PB = NQ == 1 ? 16 : 32 / NQ;                   // bytes per piece
    constexpr int IPP = PB / (int)(sizeof(AT) * T::KPL);         // instructions per piece
    typedef typename Piece<PB>::type piece_t;
    auto read_piece = [&](int buf, int q, piece_t (&fa)[WTM], piece_t (&fb)[WTN]) {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
            fa[i] = *reinterpret_cast<const piece_t*>(As[buf] + (wr * WTM * 16 + i * 16 + li) * ROW_STRIDE + lg * 32 + q * PB);
#pragma unroll
        for (int j = 0; j < WTN; ++j)
            fb[j] = *reinterpret_cast<const piece_t*>(Bs[buf] + (wc * WTN * 16 + j * 16 + li) * ROW_STRIDE + lg * 32 + q * PB);
    };
    auto mma_piece = [&](const piece_t (&fa)[WTM], const piece_t (&fb)[WTN]) {
#pragma unroll
        for (int s = 0; s < IPP; ++s)
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int j = 0; j < WTN; ++j)
                    acc[i][j] = T::mma(frag<AT>(fa[i], s), frag<AT>(fb[j], s), acc[i][j]);
    };

    load(0);
    store(0);
    __syncthreads();
    if constexpr (S::SUM32) {
        for (kidx_t kt = 0; kt < nkt; ++kt) {
            const int buf = kt & 1;
            const bool more = kt + 1 < nkt;
            if (more) load(kt + 1);
            piece_t pa[SETS][WTM], pb[SETS][WTN];
            // lgkmcnt(0), already met after the previous barrier: it tells
            // the compiler no scalar load is outstanding at the top of the
            // loop, so the waits for piece 0's reads count them one by one
            // instead of waiting for all of them
            __builtin_amdgcn_s_waitcnt(0xc07f);
            read_piece(buf, 0, pa[0], pb[0]);
            // piece 0's reads stay apart from piece 1's (not merged into
            // wider reads), so its first instructions wait for their own
            // operands only
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if constexpr (SETS == 2) {
                    if (q + 1 < NQ) read_piece(buf, q + 1, pa[(q + 1) & 1], pb[(q + 1) & 1]);
                } else {
                    if (q > 0) read_piece(buf, q, pa[0], pb[0]);
                }
                mma_piece(pa[q % SETS], pb[q % SETS]);
                // the other buffer held stage kt - 1, which every wave
                // finished reading before the previous barrier.  Float32
                // writes it after the first piece (141.1 against 139.8
                // TFLOP/s after the last at n = 50,000); bfloat16 after the
                // last (1,180 against 1,090), as does the float64 product.
                if (q == (SETS == 2 ? 0 : NQ - 1) && more) store(buf ^ 1);
                // one piece's reads and instructions at a time
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
        }
    } else if constexpr (NQ == 1) {
        for (kidx_t kt = 0; kt < nkt; ++kt) {
            const int buf = kt & 1;
            const bool more = kt + 1 < nkt;
            if (more) load(kt + 1);
            piece_t fa[2][WTM], fb[2][WTN];
            read_piece(buf, 0, fa[0], fb[0]);
            read_piece(buf, 1, fa[1], fb[1]);
            mma_piece(fa[0], fb[0]);
            mma_piece(fa[1], fb[1]);
            if constexpr (SUM64) {
                if ((kt + 1) % FLUSH_STAGES == 0 || !more) flush();
            }
            // the other buffer held stage kt - 1, which every wave finished
            // reading before the previous barrier
            if (more) store(buf ^ 1);
            __syncthreads();
        }
    } else {
        piece_t pa[2][WTM], pb[2][WTN];
        read_piece(0, 0, pa[0], pb[0]);
        for (kidx_t kt = 0; kt < nkt; ++kt) {
            const int buf = kt & 1;
            const bool more = kt + 1 < nkt;
            if (more) load(kt + 1);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (q + 1 < NQ) {
                    read_piece(buf, q + 1, pa[(q + 1) & 1], pb[(q + 1) & 1]);
                } else {
                    // the other buffer held stage kt - 1, which every wave
                    // finished reading before the previous barrier
                    if (more) store(buf ^ 1);
                    if constexpr (SUM64) {
                        if (kt % FLUSH_STAGES == FLUSH_STAGES - 1) flush();
                    }
                    __syncthreads();
                    if (more) read_piece(buf ^ 1, 0, pa[0], pb[0]);
                }
                mma_piece(pa[q & 1], pb[q & 1]);
            }
        }
        if constexpr (SUM64) flush();
    }

    // Epilogue: per column, sums over this wave's WTM*16 rows.  Rows of lane
    // (i, v): r0 + wr*WTM*16 + i*16 + ROW_G*lg + ROW_V*v; columns:
    // c0 + wc*WTN*16 + j*16 + li.
    const int Q = a.with_cross ? a.Qc + 1 : 1;
    const int64_t rw = r0 + wr * WTM * 16;
    const int64_t pb = rw / (WTM * 16);
    const int64_t cbase = c0 + wc * WTN * 16 + li;
    if constexpr (S::SUM32) {
        // one column block at a time: its values in float64 (32 registers)
        // rather than all of them at once (256)
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
            double z[WTM][4];
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) z[i][v] = (double)acc[i][j][v];
            const int64_t col = cbase + j * 16;
            if (a.with_cross) {
                for (int q = 0; q < a.Qc; ++q) {
                    const double* Cq = a.C + q * a.ldc + rw + T::ROW_G * lg;
                    double sum = 0.0;
#pragma unroll
                    for (int i = 0; i < WTM; ++i)
#pragma unroll
                        for (int v = 0; v < 4; ++v) sum += z[i][v] * Cq[i * 16 + T::ROW_V * v];
                    sum = wave_sum16(sum);
                    if (lg == 0 && col < a.cols) a.part[(pb * Q + q) * a.ldp + col] = sum;
                }
            }
            double sum = 0.0;
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) sum += z[i][v] * z[i][v];
            sum = wave_sum16(sum);
            if (lg == 0 && col < a.cols) a.part[(pb * Q + Q - 1) * a.ldp + col] = sum;
        }
        return;
    }
    if (a.with_cross) {
        for (int q = 0; q < a.Qc; ++q) {
            const double* Cq = a.C + q * a.ldc + rw + T::ROW_G * lg;
            double cv[WTM][4];
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) cv[i][v] = Cq[i * 16 + T::ROW_V * v];
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
                double sum = 0.0;
#pragma unroll
                for (int i = 0; i < WTM; ++i)
#pragma unroll
                    for (int v = 0; v < 4; ++v) sum += zval(i, j, v) * cv[i][v];
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
        for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) sum += zval(i, j, v) * zval(i, j, v);
        sum = wave_sum16(sum);
        const int64_t col = cbase + j * 16;
        if (lg == 0 && col < a.cols) a.part[(pb * Q + Q - 1) * a.ldp + col] = sum;
    }
}

// Float64 product with int8 dosages, its operands loaded straight from
// global memory into three LDS buffers: the loads of stage kt + 2 are
// issued at the top of stage kt and the end of stage kt waits only for
// stage kt + 1's (explicit vmcnt waits and a bare s_barrier, as in the
// paired-digit int8 product), so two stages of matrix instructions cover
// their latency and no staging registers or LDS writes are spent on them.
// A stage is 16 elements of K (128 bytes of a row of L^-1, 16 bytes of a
// dosage column).  L^-1 rows sit unpadded in groups of 8 rows (1 KB, one
// load instruction); chunk c of row r of a group goes to slot
// 16 (c / 2) + 8 ((c % 2) xor (group parity)) + r % 8, so a fragment read
// (16 rows, one chunk) hits distinct banks whether the LDS serves 8 or 16
// lanes of a 16-byte read per cycle.  Dosage columns keep their 16 int8
// bytes per stage side by side (a lane's four bytes per 16-column block are
// one conflict-free 4-byte read) and become float64 in registers.  Rows at
// or past n (identity rows of the padded L^-1 meet whatever follows a
// column past n) are zeroed before the sums.  The tile and the partial-sum
// layout are those of the 128 x 128 shape of 32 x 64 waves.
//
// With float64 dosages (XT = double) the dosage columns take the layout of
// the rows of L^-1 (128 bytes a stage, groups of 8 columns, the same
// swizzle), a stage holds 32 KB, and two buffers (loads one stage ahead)
// keep two workgroups per CU; elements k >= n of the last stage are zeroed
// in registers, since the bytes past a column's n belong to whatever
// follows it.
__device__ __forceinline__ int f64_slot(int r8, int c, int parity) {
    return (c >> 1) * 16 + (((c & 1) ^ parity) << 3) + r8;
}

template <typename XT, bool GROUPED>
__global__ __launch_bounds__(512, sizeof(XT) == 8 ? 4 : 2) void trmm_f64_lds_kernel(TrmmArgs la) {
    typedef MM<double> T;
    constexpr bool XD = sizeof(XT) == 8;
    constexpr int NBUF = XD ? 2 : 3, LOOK = NBUF - 1;
    constexpr int WGM = 4, WGN = 2, WTM = 2, WTN = 4;
    constexpr int TM = WGM * WTM * 16, TN = WGN * WTN * 16, NW = WGM * WGN;
    constexpr int BK = 16;                         // K per stage
    constexpr int AB = TM * BK * 8;                // bytes of L^-1 per stage buffer
    constexpr int XBB = TN * BK * (int)sizeof(XT); // bytes of dosages per stage buffer
    // load instructions per stage (1 KB each): L^-1, dosages
    constexpr int NA = TM / 8, NB = XD ? TN / 8 : TN / 64;
    static_assert(NA % NW == 0 && (XD ? NB % NW == 0 : NB <= NW), "load instructions per wave");
    constexpr int LA = NA / NW;
    // s_waitcnt immediates: vmcnt(this wave's loads per stage) or vmcnt(0),
    // with lgkmcnt(0) and any expcnt; waves below NB issue one dosage load
    constexpr int WAIT_MORE = (LA + 1) | (7 << 4);
    constexpr int WAIT_LESS = LA | (7 << 4);
    constexpr int WAIT_ALL = 7 << 4;

    const int e0 = __builtin_amdgcn_readfirstlane(la.sched[2 * (int64_t)blockIdx.x]);
    const int J = __builtin_amdgcn_readfirstlane(la.sched[2 * (int64_t)blockIdx.x + 1]);
    if (e0 < 0) return;
    const int I = e0 & SCHED_ROW_MASK;
    const TrmmArgs a = GROUPED ? la.group[e0 >> SCHED_CTX_SHIFT] : la;
    if ((int64_t)J * TN >= a.cols) return;

    __shared__ __attribute__((aligned(1024))) char Abuf[NBUF][AB];
    __shared__ __attribute__((aligned(1024))) char Bbuf[NBUF][XBB];
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

    const int64_t r0 = (int64_t)I * TM;
    const int64_t c0 = (int64_t)J * TN;
    const int64_t kend = a.full_k ? a.n_pad : std::min<int64_t>(r0 + TM, a.n_pad);
    const int nk = (int)(kend / BK);
    const int64_t row_bytes = a.ldu * 8;

    const u4_t rsA = buffer_words(reinterpret_cast<const char*>(a.Ut) + r0 * row_bytes, (uint32_t)(TM * row_bytes));
    const int64_t xcols = std::min<int64_t>(TN, a.cols - c0);
    const int64_t xbytes = (((xcols - 1) * a.ldx + a.n) * (int64_t)sizeof(XT) + 15) / 16 * 16;
    const u4_t rsB = buffer_words(reinterpret_cast<const char*>(a.X) + c0 * a.ldx * (int64_t)sizeof(XT),
                                  (uint32_t)xbytes);
    // lane l of an L^-1 load instruction (group q of 8 rows) fetches the
    // chunk that belongs in slot l; lane l of an int8 dosage load, column l
    // of its 64 (float64 dosages: as L^-1, groups of 8 columns)
    const int lr8 = lane & 7;
    const int lc_even = 2 * (lane >> 4) + ((lane >> 3) & 1);       // chunk for an even group
    const int lc_odd = 2 * (lane >> 4) + (((lane >> 3) & 1) ^ 1);  // chunk for an odd group
    const bool has_b = wave < NB;
    auto load = [&](int kt, char* Ab, char* Bb) {
#pragma unroll
        for (int c = 0; c < LA; ++c) {
            const int q = wave + c * NW;
            const int ch = (q & 1) ? lc_odd : lc_even;
            load_lds16(rsA, lds_address(Ab + q * 1024),
                       (uint32_t)((q * 8 + lr8) * row_bytes + kt * (BK * 8) + ch * 16));
        }
        if constexpr (XD) {
#pragma unroll
            for (int c = 0; c < NB / NW; ++c) {
                const int q = wave + c * NW;
                const int ch = (q & 1) ? lc_odd : lc_even;
                load_lds16(rsB, lds_address(Bb + q * 1024),
                           (uint32_t)((q * 8 + lr8) * a.ldx * 8 + kt * (BK * 8) + ch * 16));
            }
        } else if (has_b) {
            load_lds16(rsB, lds_address(Bb + wave * 1024), (uint32_t)((wave * 64 + lane) * a.ldx + kt * BK));
        }
    };

    d4_t acc[WTM][WTN];
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    // this lane's fragment addresses within a stage buffer: rows
    // wr*32 + i*16 + li, chunks 2 lg and 2 lg + 1; dosage bytes 4 lg.. of
    // columns wc*64 + j*16 + li
    int aoff[WTM][2];
#pragma unroll
    for (int i = 0; i < WTM; ++i) {
        const int row = wr * WTM * 16 + i * 16 + li;
#pragma unroll
        for (int h = 0; h < 2; ++h) aoff[i][h] = (row >> 3) * 1024 + f64_slot(row & 7, 2 * lg + h, (row >> 3) & 1) * 16;
    }
    const int boff = (wc * WTN * 16 + li) * BK + lg * 4;
    int boffd[WTN][2];                   // float64 dosages: columns laid out as rows of L^-1
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
        const int col = wc * WTN * 16 + j * 16 + li;
#pragma unroll
        for (int h = 0; h < 2; ++h) boffd[j][h] = (col >> 3) * 1024 + f64_slot(col & 7, 2 * lg + h, (col >> 3) & 1) * 16;
    }

    auto stage = [&](int kt, const char* Ar, const char* Br, char* An, char* Bn) {
        const bool ahead = kt + LOOK < nk;
        if (ahead) load(kt + LOOK, An, Bn);
        if constexpr (XD) {
            // float64 dosages: K = 16 kt + 4 lg + st at or past n reads as
            // zero; one 16-byte piece (two K) of each fragment at a time
            const int kl = (int)a.n - (kt * BK + 4 * lg);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                u4_t fa[WTM], fd[WTN];
#pragma unroll
                for (int i = 0; i < WTM; ++i) fa[i] = *reinterpret_cast<const u4_t*>(Ar + aoff[i][h]);
#pragma unroll
                for (int j = 0; j < WTN; ++j) fd[j] = *reinterpret_cast<const u4_t*>(Br + boffd[j][h]);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int st = 2 * h + e;
                    double xb[WTN];
#pragma unroll
                    for (int j = 0; j < WTN; ++j) {
                        const u2_t x2 = e ? u2_t{fd[j][2], fd[j][3]} : u2_t{fd[j][0], fd[j][1]};
                        xb[j] = st < kl ? __builtin_bit_cast(double, x2) : 0.0;
                    }
#pragma unroll
                    for (int i = 0; i < WTM; ++i) {
                        const u2_t w2 = e ? u2_t{fa[i][2], fa[i][3]} : u2_t{fa[i][0], fa[i][1]};
                        const double av = __builtin_bit_cast(double, w2);
#pragma unroll
                        for (int j = 0; j < WTN; ++j) acc[i][j] = T::mma(av, xb[j], acc[i][j]);
                    }
                }
            }
        } else {
            u4_t fa[WTM][2];
            uint32_t fb[WTN];
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int h = 0; h < 2; ++h) fa[i][h] = *reinterpret_cast<const u4_t*>(Ar + aoff[i][h]);
#pragma unroll
            for (int j = 0; j < WTN; ++j) fb[j] = *reinterpret_cast<const uint32_t*>(Br + boff + j * 16 * BK);
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                double xb[WTN];
#pragma unroll
                for (int j = 0; j < WTN; ++j) xb[j] = (double)(int)(int8_t)(fb[j] >> (8 * st));
#pragma unroll
                for (int i = 0; i < WTM; ++i) {
                    const u2_t w2 = (st & 1) ? u2_t{fa[i][st >> 1][2], fa[i][st >> 1][3]}
                                             : u2_t{fa[i][st >> 1][0], fa[i][st >> 1][1]};
                    const double av = __builtin_bit_cast(double, w2);
#pragma unroll
                    for (int j = 0; j < WTN; ++j) acc[i][j] = T::mma(av, xb[j], acc[i][j]);
                }
            }
        }
        // the stage's matrix instructions stay ahead of its barrier
        __builtin_amdgcn_sched_barrier(0);
        // three buffers: wait only for stage kt + 1 (kt + 2 stays in
        // flight); two: for everything
        if (LOOK == 1 || !ahead) __builtin_amdgcn_s_waitcnt(WAIT_ALL);
        else if (has_b) __builtin_amdgcn_s_waitcnt(WAIT_MORE);
        else __builtin_amdgcn_s_waitcnt(WAIT_LESS);
        compiler_fence();
        __builtin_amdgcn_s_barrier();
        compiler_fence();
    };

    load(0, A0, B0);
    if (LOOK == 2 && nk > 1) {
        load(1, A1, B1);
        if (has_b) __builtin_amdgcn_s_waitcnt(WAIT_MORE);
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

    // Epilogue (as the staged float64 tiles): per column, sums over this
    // wave's 32 rows; rows at or past n are zeroed first
    const int Q = a.with_cross ? a.Qc + 1 : 1;
    const int64_t rw = r0 + wr * WTM * 16;
    const int64_t pb = rw / (WTM * 16);
    const int64_t cbase = c0 + wc * WTN * 16 + li;
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (rw + i * 16 + T::ROW_G * lg + T::ROW_V * v >= a.n)
#pragma unroll
                for (int j = 0; j < WTN; ++j) acc[i][j][v] = 0.0;
    if (a.with_cross) {
        for (int q = 0; q < a.Qc; ++q) {
            const double* Cq = a.C + q * a.ldc + rw + T::ROW_G * lg;
            double cv[WTM][4];
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) cv[i][v] = Cq[i * 16 + T::ROW_V * v];
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
                double sum = 0.0;
#pragma unroll
                for (int i = 0; i < WTM; ++i)
#pragma unroll
                    for (int v = 0; v < 4; ++v) sum += acc[i][j][v] * cv[i][v];
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
        for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) sum += acc[i][j][v] * acc[i][j][v];
        sum = wave_sum16(sum);
        const int64_t col = cbase + j * 16;
        if (lg == 0 && col < a.cols) a.part[(pb * Q + Q - 1) * a.ldp + col] = sum;
    }
}

// Tile shapes of the triangular product.  MINB is the workgroups per CU
// the register budget is sized for.
typedef Shape<2, 2, 4, 4, 2> Cfg0;   // 128 x 128, 256 threads, waves of 64 x 64
typedef Shape<2, 4, 4, 2, 1> Cfg1;   // 128 x 128, 512 threads, waves of 64 x 32
typedef Shape<4, 2, 2, 4, 1> Cfg2;   // 128 x 128, 512 threads, waves of 32 x 64
typedef Shape<2, 4, 4, 4, 1> Cfg3;   // 128 x 256, 512 threads, waves of 64 x 64
typedef Shape<4, 2, 4, 4, 1> Cfg4;   // 256 x 128, 512 threads, waves of 64 x 64
typedef Shape<2, 2, 4, 4, 1> Cfg5;   // as Cfg0, one workgroup per CU
typedef Shape<4, 2, 4, 8, 1, true> Cfg6;   // 256 x 256, 512 threads, waves of 64 x 128, float32 sums

template <typename S> TrmmShape shape_of() { return TrmmShape{S::TM, S::TN, S::WTM * 16, S::NT, 1, 32}; }

template <typename AT, typename XT, typename S>
hipError_t launch_trmm(const TrmmArgs& a, hipStream_t s) {
    if (a.group)
        hipLaunchKernelGGL((trmm_stream_kernel<AT, XT, S, true>), dim3((unsigned)a.n_sched), dim3(S::NT), 0, s, a);
    else
        hipLaunchKernelGGL((trmm_stream_kernel<AT, XT, S, false>), dim3((unsigned)a.n_sched), dim3(S::NT), 0, s, a);
    return hipGetLastError();
}

template <typename AT, typename XT>
hipError_t launch_cfg(const TrmmArgs& a, hipStream_t s) {
    // only the shapes trmm_cfg_valid admits are instantiated
    constexpr bool F64 = sizeof(AT) == 8;
    constexpr bool I8 = sizeof(XT) == 1;
    switch (a.cfg) {
        case 1: return launch_trmm<AT, XT, Cfg1>(a, s);
        case 2: return launch_trmm<AT, XT, Cfg2>(a, s);
        case 5: return launch_trmm<AT, XT, Cfg5>(a, s);
        case 3:
            if constexpr (F64 || I8) return launch_trmm<AT, XT, Cfg3>(a, s);
            else return hipErrorInvalidValue;
        case 0:
            if constexpr (F64) return launch_trmm<AT, XT, Cfg0>(a, s);
            else return hipErrorInvalidValue;
        case 4:
            if constexpr (F64) return launch_trmm<AT, XT, Cfg4>(a, s);
            else return hipErrorInvalidValue;
        case 6:
            if constexpr (!F64 && (I8 || std::is_same<XT, __bf16>::value)) return launch_trmm<AT, XT, Cfg6>(a, s);
            else return hipErrorInvalidValue;
        case 7:
            if constexpr (F64 && I8) {
                if (a.group)
                    hipLaunchKernelGGL((trmm_f64_lds_kernel<int8_t, true>), dim3((unsigned)a.n_sched), dim3(512), 0, s, a);
                else
                    hipLaunchKernelGGL((trmm_f64_lds_kernel<int8_t, false>), dim3((unsigned)a.n_sched), dim3(512), 0, s, a);
                return hipGetLastError();
            } else if constexpr (F64) {
                if (a.group)
                    hipLaunchKernelGGL((trmm_f64_lds_kernel<double, true>), dim3((unsigned)a.n_sched), dim3(512), 0, s, a);
                else
                    hipLaunchKernelGGL((trmm_f64_lds_kernel<double, false>), dim3((unsigned)a.n_sched), dim3(512), 0, s, a);
                return hipGetLastError();
            } else {
                return hipErrorInvalidValue;
            }
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int trmm_num_cfgs() { return 8; }
int trmm_cfg_limit() { return std::max(trmm_num_cfgs(), trmm_sliced_cfgs()); }

bool trmm_shape_sum32(int cfg) { return cfg == 6; }

TrmmShape trmm_shape(int cfg) {
    switch (cfg) {
        case 0: return shape_of<Cfg0>();
        case 1: return shape_of<Cfg1>();
        case 2: return shape_of<Cfg2>();
        case 3: return shape_of<Cfg3>();
        case 4: return shape_of<Cfg4>();
        case 5: return shape_of<Cfg5>();
        case 6: return shape_of<Cfg6>();
        case 7: return shape_of<Cfg2>();   // the float64 direct-load kernel: Cfg2's tile
        default: return TrmmShape{0, 0, 0, 0, 0, 0};
    }
}

bool trmm_cfg_valid(int at, int xt, int cfg) {
    if (at == A_I8S) return xt == X_I8 && cfg >= 0 && cfg < trmm_sliced_cfgs();
    if (cfg < 0 || cfg >= trmm_num_cfgs()) return false;
    // bfloat16 slices of float64 dosages feed the bfloat16 product only
    if ((xt == X_BF16S || xt == X_BF16) && at != A_BF16) return false;
    // 64 x 128 waves fit two per SIMD only with float32 sums and one- or
    // two-byte dosages
    if (cfg == 6) return at != A_F64 && (xt == X_I8 || xt == X_BF16S || xt == X_BF16);
    // float64 loaded straight into LDS
    if (cfg == 7) return at == A_F64;
    if (at == A_F64) return true;
    // The reduced-precision products also carry float64 partial sums; 64 x 64
    // waves of them only fit two waves per SIMD without spilling when the
    // staged dosages are int8 and the tile is 128 x 256.
    if (cfg == 1 || cfg == 2 || cfg == 5) return true;
    return cfg == 3 && xt == X_I8;
}

// Measured on MI355X at n = 50,000 with int8 dosages (one 50,000-SNP block):
// float64 is fastest in the 128 x 128 tile of 32 x 64 waves (67.5 TFLOP/s,
// against 66.0 in the 128 x 256 tile, 67.3 in the 256 x 128 tile), and
// that tile a little faster again with its operands loaded straight into
// LDS (shape 7: 67.8 against 67.35 TFLOP/s in the same run); float32
// and bfloat16 in the 256 x 256 tile of 64 x 128 waves with float32 sums
// (141 and 1,180 TFLOP/s, against 131 and 870 in the 128 x 256 tile with
// float64 sums; b moves from 6e-11 to 4e-10 of the float64 path for
// float32, and not measurably for bfloat16, whose rounding of L^-1
// dominates).  With float64 dosages the float64 product is faster loaded
// straight into LDS too (shape 7 against the 128 x 256 register-staged
// tile: 0.845 against 0.804 of peak at n = 50,000, 0.753 against 0.707 at
// n = 20,000 in calls of 5,000 SNPs), and the reduced-precision products
// take the 128 x 128 tile of 64 x 32 waves.
int trmm_default_cfg(int at, int xt) {
    if (at == A_I8S) return trmm_sliced_default_cfg();
    if (at == A_F64) return 7;
    if (xt == X_I8 || xt == X_BF16S || xt == X_BF16) return 6;
    return 1;
}

TrmmShape trmm_geom(int at, int xt, int cfg, int slices, int rgroup) {
    TrmmShape sh = (at == A_I8S) ? trmm_sliced_shape(cfg) : trmm_shape(cfg);
    if (sh.tm == 0) return sh;
    // workgroups per CU: the 256-thread shape and the float64 direct-load
    // shape are sized for two
    const int per_cu = (at != A_I8S && (cfg == 0 || cfg == 7)) || (at == A_I8S && trmm_sliced_two_per_cu(cfg)) ? 2 : 1;
    sh.inflight = 32 * per_cu;
    const int64_t asz = at == A_F64 ? 8 : at == A_F32 ? 4 : at == A_BF16 ? 2 : 1;
    const int64_t arows = at == A_I8S ? (int64_t)sh.tm * slices : sh.tm;
    const int64_t xsz = x_elem_bytes(xt);
    sh.rgroup = rgroup > 0 ? std::min(rgroup, sh.inflight)
                           : row_group_for(arows * asz, (int64_t)sh.tn * xsz, sh.inflight);
    return sh;
}

int64_t trmm_schedule_len(int64_t n_pad, int64_t cols, const TrmmShape& sh) {
    const int64_t nrb = n_pad / sh.tm;
    return trmm_schedule_multi(&nrb, 1, cols, sh, nullptr);
}

int64_t trmm_schedule(int64_t n_pad, int64_t cols, const TrmmShape& sh, int* out, int64_t cap) {
    const int64_t nrb = n_pad / sh.tm;
    std::vector<int> v;
    const int64_t total = trmm_schedule_multi(&nrb, 1, cols, sh, &v);
    if (total > cap) return -1;
    std::copy(v.begin(), v.end(), out);
    return total;
}

hipError_t trmm_check(const TrmmArgs& a, bool check_sched) {
    if (a.cols <= 0) return hipSuccess;
    if (!a.Ut || !a.X || !a.part || !a.sched) return hipErrorInvalidValue;
    if (a.n_pad % NPAD_ALIGN || a.ldu < a.n_pad || a.n > a.n_pad || a.n < 1) return hipErrorInvalidValue;
    if (a.ldx < a.n || a.ldp < a.cols) return hipErrorInvalidValue;
    if (a.with_cross && (!a.C || a.ldc < a.n_pad || a.Qc < 1)) return hipErrorInvalidValue;
    const size_t xs = (size_t)x_elem_bytes(a.xt);
    if ((reinterpret_cast<uintptr_t>(a.X) % 16) || ((a.ldx * xs) % 16)) return hipErrorInvalidValue;
    // bfloat16 dosage slices: three per column, n_pad elements each
    if (a.xt == X_BF16S && (a.at != A_BF16 || a.slices != 3 || a.ldx < 3 * a.n_pad)) return hipErrorInvalidValue;
    if (a.xt == X_BF16 && (a.at != A_BF16 || a.slices == 3 || a.ldx < a.n_pad)) return hipErrorInvalidValue;
    if (a.at == A_I8S) {
        // the int8-slice product forms z^T z only (its mode takes the cross
        // products from x^T W)
        if (!a.rscale || !a.rsum || a.xt != X_I8 || (a.ldu % 16) || a.slices < 4 || a.slices > 6 || a.with_cross ||
            a.n_pad >= (1 << 18) ||
            !trmm_cfg_valid(a.at, a.xt, a.cfg))
            return hipErrorInvalidValue;
        // 32-bit buffer offsets of the shapes that load straight into LDS
        const TrmmShape sh = trmm_sliced_shape(a.cfg);
        if (trmm_sliced_direct(a.cfg) &&
            ((int64_t)sh.tm * a.slices * a.ldu > INT32_MAX || (int64_t)sh.tn * a.ldx + a.n_pad > INT32_MAX))
            return hipErrorInvalidValue;
    } else {
        if (!trmm_cfg_valid(a.at, a.xt, a.cfg)) return hipErrorInvalidValue;
    }
    const TrmmShape sh = trmm_geom(a.at, a.xt, a.cfg, a.slices, a.rgroup);
    if (a.n_pad % sh.tm) return hipErrorInvalidValue;
    // 32-bit buffer offsets of the SUM32 shapes and of the float64
    // direct-load shape: a tile's rows of L^-1 and its dosage columns up to
    // the last stage
    if (a.at != A_I8S && (trmm_shape_sum32(a.cfg) || a.cfg == 7)) {
        const int64_t asz = a.at == A_F64 ? 8 : a.at == A_F32 ? 4 : 2;
        if ((int64_t)sh.tm * a.ldu * asz > INT32_MAX || ((int64_t)sh.tn * a.ldx + a.n_pad) * (int64_t)xs > INT32_MAX)
            return hipErrorInvalidValue;
    }
    const int64_t scols = a.sched_cols ? a.sched_cols : a.cols;
    if (scols < a.cols) return hipErrorInvalidValue;
    if (check_sched && (a.n_sched != trmm_schedule_len(a.n_pad, scols, sh)))
        return hipErrorInvalidValue;
    if (a.n_sched > 0x7fffffff) return hipErrorInvalidValue;
    return hipSuccess;
}

// Single launches check their own arguments; grouped launches (a.group set)
// have had every context's arguments checked by the caller with trmm_check.
hipError_t trmm_stream(const TrmmArgs& a, hipStream_t s) {
    if (a.cols <= 0 && !a.group) return hipSuccess;
    if (!a.group) {
        hipError_t e = trmm_check(a, true);
        if (e != hipSuccess) return e;
    } else if (!a.sched || a.n_sched <= 0 || a.n_sched > 0x7fffffff) {
        return hipErrorInvalidValue;
    }
    if (a.at == A_I8S) return trmm_sliced_launch(a, s);
    if (a.xt == X_F64) {
        if (a.at == A_F64) return launch_cfg<double, double>(a, s);
        if (a.at == A_F32) return launch_cfg<float, double>(a, s);
        if (a.at == A_BF16) return launch_cfg<__bf16, double>(a, s);
    } else if (a.xt == X_BF16S || a.xt == X_BF16) {
        if (a.at == A_BF16) return launch_cfg<__bf16, __bf16>(a, s);
    } else if (a.xt == X_I8) {
        if (a.at == A_F64) return launch_cfg<double, int8_t>(a, s);
        if (a.at == A_F32) return launch_cfg<float, int8_t>(a, s);
        if (a.at == A_BF16) return launch_cfg<__bf16, int8_t>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gwas
