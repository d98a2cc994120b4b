// vmc_mfma.hpp -- 16x16x4 matrix-core products in FP64 and FP32 (gfx950).
//
// Operand layouts of v_mfma_{f64,f32}_16x16x4 (one wavefront, lane l):
//   A: lane l supplies A[l % 16][l / 16]   (row, k)
//   B: lane l supplies B[l / 16][l % 16]   (k, column)
//   D: register v of lane l holds D[row(l, v)][l % 16] with
//      row = l / 16 + 4 v (FP64)  or  4 (l / 16) + v (FP32).
#pragma once

#include <hip/hip_runtime.h>

namespace vmcx {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    typedef v4d acc_t;
    __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc_t fma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int l, int v) { return (l >> 4) + 4 * v; }
};

template <>
struct Mfma<float> {
    typedef v4f acc_t;
    __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
    __device__ static acc_t fma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};

}  // namespace vmcx
