// Matrix-core (MFMA) product types of the M2L kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace tdbem {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<double> {
    typedef v4d acc_t;
    __device__ static acc_t op(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }      // output layout of the f64 form
};
template <> struct Mma<float> {
    typedef v4f acc_t;
    __device__ static acc_t op(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }      // output layout of the f32 form
};


}  // namespace tdbem
