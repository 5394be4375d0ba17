// Sustained matrix-core rate of the instruction each product mode runs,
// measured at the clock the device holds under that load.  Every wave of a
// launch that fills the chip issues a long run of independent 16 x 16
// instructions on register operands; the rate is instructions x their
// operations / elapsed time.  It is the measured counterpart of the
// published peak that the triangular product's fraction of peak is quoted
// against.
#include <hip/hip_runtime.h>

#include "gwas.h"

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef int i4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int GRID = 4;             // GRID x GRID independent accumulators per wave
constexpr int CHAINS = GRID * GRID;
constexpr int PROBE_THREADS = 256;
constexpr int PROBE_BLOCKS = 2048;  // 8 workgroups of 4 waves per CU on 256 CUs

// The loop has the shape of the triangular product's inner step: GRID
// operands of A and of B, every pair multiplied into its own accumulator.
template <typename Op, typename Acc, typename F>
__device__ __forceinline__ double run(const Op (&a)[GRID], const Op (&b)[GRID], int64_t iters, F mma) {
    Acc acc[GRID][GRID];
#pragma unroll
    for (int i = 0; i < GRID; ++i)
#pragma unroll
        for (int j = 0; j < GRID; ++j) acc[i][j] = Acc{0, 0, 0, 0};
    for (int64_t k = 0; k < iters; ++k)
#pragma unroll
        for (int i = 0; i < GRID; ++i)
#pragma unroll
            for (int j = 0; j < GRID; ++j) acc[i][j] = mma(a[i], b[j], acc[i][j]);
    double out = 0.0;
#pragma unroll
    for (int i = 0; i < GRID; ++i)
#pragma unroll
        for (int j = 0; j < GRID; ++j) out += (double)acc[i][j][0] + (double)acc[i][j][3];
    return out;
}

template <int KIND>
__global__ __launch_bounds__(PROBE_THREADS) void peak_kernel(int64_t iters, double* sink) {
    const int t = threadIdx.x;
    double out = 0.0;
    if constexpr (KIND == GWAS_FP64) {
        double a[GRID], b[GRID];
        for (int i = 0; i < GRID; ++i) {
            a[i] = 1.0 + (t + i) * 1e-9;
            b[i] = 1.0 - (t + i) * 1e-9;
        }
        out = run<double, d4_t>(a, b, iters, [](double x, double y, d4_t c) {
            return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
        });
    } else if constexpr (KIND == GWAS_FP32_REFINE) {
        float a[GRID], b[GRID];
        for (int i = 0; i < GRID; ++i) {
            a[i] = 1.0f + (t + i) * 1e-6f;
            b[i] = 1.0f - (t + i) * 1e-6f;
        }
        out = run<float, f4_t>(a, b, iters, [](float x, float y, f4_t c) {
            return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
        });
    } else if constexpr (KIND == GWAS_BF16_REFINE) {
        bf8_t a[GRID], b[GRID];
        for (int i = 0; i < GRID; ++i)
            for (int e = 0; e < 8; ++e) {
                a[i][e] = (__bf16)(1.0f + (t + i + e) * 1e-3f);
                b[i][e] = (__bf16)(1.0f - (t + i + e) * 1e-3f);
            }
        out = run<bf8_t, f4_t>(a, b, iters, [](bf8_t x, bf8_t y, f4_t c) {
            return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
        });
    } else {
        i4_t a[GRID], b[GRID];
        for (int i = 0; i < GRID; ++i) {
            a[i] = i4_t{t + i, t + i + 1, t + i + 2, t + i + 3} & 0x01010101;
            b[i] = i4_t{1, 1, 1, 1} << i;
        }
        out = run<i4_t, i4_t>(a, b, iters, [](i4_t x, i4_t y, i4_t c) {
            return __builtin_amdgcn_mfma_i32_16x16x64_i8(x, y, c, 0, 0, 0);
        });
    }
    sink[(int64_t)blockIdx.x * PROBE_THREADS + t] = out;
}

// operations of one instruction: 2 * 16 * 16 * K
double ops_per_inst(int kind) {
    switch (kind) {
        case GWAS_FP64: return 2.0 * 16 * 16 * 4;
        case GWAS_FP32_REFINE: return 2.0 * 16 * 16 * 4;
        case GWAS_BF16_REFINE: return 2.0 * 16 * 16 * 32;
        default: return 2.0 * 16 * 16 * 64;
    }
}

hipError_t launch(int kind, int64_t iters, double* sink, hipStream_t s) {
    const dim3 g(PROBE_BLOCKS), b(PROBE_THREADS);
    switch (kind) {
        case GWAS_FP64: hipLaunchKernelGGL(peak_kernel<GWAS_FP64>, g, b, 0, s, iters, sink); break;
        case GWAS_FP32_REFINE: hipLaunchKernelGGL(peak_kernel<GWAS_FP32_REFINE>, g, b, 0, s, iters, sink); break;
        case GWAS_BF16_REFINE: hipLaunchKernelGGL(peak_kernel<GWAS_BF16_REFINE>, g, b, 0, s, iters, sink); break;
        default: hipLaunchKernelGGL(peak_kernel<GWAS_INT8_SLICED>, g, b, 0, s, iters, sink); break;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" int gwas_peak_probe(int32_t kind, int32_t device, int64_t iters, double* ops_per_s) {
    if (!ops_per_s || kind < GWAS_FP64 || kind > GWAS_INT8_SLICED || iters < 1 || iters > (1LL << 32))
        return GWAS_E_INVALID;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return GWAS_E_NO_DEVICE;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return GWAS_E_HIP;
    if (hipSetDevice(device) != hipSuccess) return GWAS_E_NO_DEVICE;
    int rc = GWAS_OK;
    double* sink = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
    if (hipMalloc((void**)&sink, sizeof(double) * PROBE_BLOCKS * PROBE_THREADS) != hipSuccess) {
        rc = GWAS_E_OOM;
    } else if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
               hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
               launch(kind, iters, sink, s) != hipSuccess ||   // the clock settles under load
               hipEventRecord(e0, s) != hipSuccess || launch(kind, iters, sink, s) != hipSuccess ||
               hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
               hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f)) {
        rc = GWAS_E_HIP;
    }
    if (rc == GWAS_OK)
        *ops_per_s = ops_per_inst(kind) * CHAINS * (double)iters * PROBE_BLOCKS * (PROBE_THREADS / 64) /
                     (ms * 1e-3);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (sink) (void)hipFree(sink);
    (void)hipSetDevice(prev);
    (void)hipGetLastError();
    return rc;
}
