// Definitions shared by the two forms of the streaming triangular product
// (floating-point tiles and int8 slices): fragment vector types, the LDS
// stage row layout, loads straight into LDS and the lane-group reduction of
// the epilogues.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gwas {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u2_t __attribute__((ext_vector_type(2)));
typedef int i4_t __attribute__((ext_vector_type(4)));

// Each LDS row of a stage holds 128 bytes of K (BK elements) plus 16 bytes of
// padding, so the 16 rows read together by one instruction fall on
// distinct banks and every row stays 16-byte aligned.
constexpr int ROW_BYTES = 128;
constexpr int ROW_STRIDE = ROW_BYTES + 16;

// Compiler-only ordering of memory operations around a stage barrier.
__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// One 16-byte-per-lane buffer load straight into LDS: lane l's 16 bytes
// land at lds + 16 l (M0 holds the instruction's LDS address).  Written out
// because the compiler, which does not follow the three buffers through the
// unrolled stage loop, would otherwise wait for every load in flight before
// the first read of a stage; the loads write no registers, and the stage
// loop orders them with explicit vmcnt waits and barriers.  Nothing else in
// the kernels using it use M0.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void load_lds16(u4_t rsrc, uint32_t lds, uint32_t voff) {
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
                 :: "s"(lds), "v"(voff), "s"(rsrc) : "memory", "m0");
}
#pragma clang diagnostic pop

// Buffer descriptor words (base, range in bytes), as for the buffer loads
// elsewhere (flags word 0x00020000), held in scalar registers.
__device__ __forceinline__ u4_t buffer_words(const void* base, uint32_t bytes) {
    const uint64_t b = reinterpret_cast<uint64_t>(base);
    u4_t r;
    r[0] = __builtin_amdgcn_readfirstlane((uint32_t)b);
    r[1] = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32) & 0xffffu);
    r[2] = __builtin_amdgcn_readfirstlane(bytes);
    r[3] = 0x00020000u;
    return r;
}

// LDS byte address of p, wave-uniform, in a scalar register
__device__ __forceinline__ uint32_t lds_address(const char* p) {
    return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char*)p);
}

__device__ __forceinline__ double wave_sum16(double v) {
    // sum over the four lane groups (lanes l, l+16, l+32, l+48)
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

}  // namespace
}  // namespace gwas
