// Layout probes of the MFMA builtins used by the kernels: one wave computes a
// single 16 x 16 product from row-major operands and writes D row-major using
// the accumulator layout the kernels assume (element i of lane l holds row
// 4*(l/16) + i, column l % 16).  Exported for the test suite.
#include "internal.hpp"
#include "xpcs_diag.h"

namespace xpcs {
namespace {

// A: 16 x 32 floats (exact in bf16), B: 32 x 16 floats; lane l feeds row/column
// l % 16 and K group l / 16 (8 consecutive K).
__global__ __launch_bounds__(64) void probe_bf16_kernel(const float *A, const float *B, double *D) {
    const int l = threadIdx.x, r = l & 15, g = l >> 4;
    u16x8 a, b;
    for (int e = 0; e < 8; ++e) {
        a[e] = f32_to_bf16_bits(A[r * 32 + 8 * g + e]);
        b[e] = f32_to_bf16_bits(B[(8 * g + e) * 16 + r]);
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma_bf16(a, b, acc);
    for (int i = 0; i < 4; ++i) D[(4 * g + i) * 16 + r] = acc[i];
}

// A: 16 x 64 int8, B: 64 x 16 int8; K groups of 16 consecutive values.
__global__ __launch_bounds__(64) void probe_i8_kernel(const int8_t *A, const int8_t *B, double *D) {
    const int l = threadIdx.x, r = l & 15, g = l >> 4;
    i32x4 a, b;
    for (int w = 0; w < 4; ++w) {
        int x = 0, y = 0;
        for (int e = 0; e < 4; ++e) {
            const int kk = 16 * g + 4 * w + e;
            x |= ((int)(uint8_t)A[r * 64 + kk]) << (8 * e);
            y |= ((int)(uint8_t)B[kk * 16 + r]) << (8 * e);
        }
        a[w] = x;
        b[w] = y;
    }
    i32x4 acc = {0, 0, 0, 0};
    acc = mfma_i8(a, b, acc);
    for (int i = 0; i < 4; ++i) D[(4 * g + i) * 16 + r] = (double)acc[i];
}

}  // namespace
}  // namespace xpcs

extern "C" {

int32_t xpcs_probe_mfma_bf16(const float *A, const float *B, double *D) {
    hipLaunchKernelGGL(xpcs::probe_bf16_kernel, dim3(1), dim3(64), 0, nullptr, A, B, D);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

int32_t xpcs_probe_mfma_i8(const int8_t *A, const int8_t *B, double *D) {
    hipLaunchKernelGGL(xpcs::probe_i8_kernel, dim3(1), dim3(64), 0, nullptr, A, B, D);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"
