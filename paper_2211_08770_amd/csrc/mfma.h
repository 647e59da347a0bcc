// 16x16x4 matrix-core (MFMA) fragments for gfx950, in FP64 and FP32.
//
// Operand layout of one 16x16x4 step (64 lanes): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; the 16x16 result D sits in four registers per lane.
// Register v of lane l holds D[row(l, v)][l%16] with
//   f64: row = 4v + l/16,   f32: row = 4(l/16) + v.
#pragma once
#include <hip/hip_runtime.h>

namespace tto {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<double> {
  typedef v4d acc_t;
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t mma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct Mma<float> {
  typedef v4f acc_t;
  __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

}  // namespace tto
