// Matrix-core operations the factorisation uses: 16x16x4 MFMA in FP64 and
// FP32 (gfx950, wave64) with their lane layouts.
#pragma once

#include "device_common.hpp"

namespace abdf {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Lane layouts of the 16x16x4 matrix-core operations (wave64):
//   A operand: lane l holds A[l % 16][l / 16];  B operand: B[l / 16][l % 16];
//   accumulator register v of lane l holds C[row(l, v)][l % 16], where the
//   FP64 form interleaves rows (row = 4 v + l / 16) and the FP32 form blocks
//   them (row = 4 (l / 16) + v).  abdf_selftest checks both on the device.
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    using acc_t = f64x4;
    __device__ static acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

template <>
struct Mfma<float> {
    using acc_t = f32x4;
    __device__ static acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

}  // namespace abdf
