// Definitions shared by the two forms of the streaming triangular product
// (floating-point tiles and int8 slices): fragment vector types, the LDS
// stage row layout and the lane-group reduction of the epilogues.
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

__device__ __forceinline__ double wave_sum16(double v) {
    // sum over the four lane groups (lanes l, l+16, l+32, l+48)
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

}  // namespace
}  // namespace gwas
