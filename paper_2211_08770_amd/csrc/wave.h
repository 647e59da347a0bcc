// Wave-level (64-lane) reductions and broadcasts for gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace tto {

// Pointers into device memory that reach a kernel inside a task descriptor are
// generic to the compiler, which then emits FLAT instructions; those count
// against the LDS wait counter too, so every LDS wait also waits for the
// global loads in flight.  glb() marks such a pointer as global memory.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __attribute__((always_inline)) inline gptr<T> glb(T* p) {
  return (gptr<T>)p;
}

// DPP move of a double within 16-lane rows (GFX9 DPP controls).
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Value of v in lane `lane` (wave-uniform result).
__device__ inline double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over each 16-lane row of a wave (every lane gets its row's sum).
__device__ inline double row16_sum(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm(1,0,3,2)
  v += dpp_d<0x4E>(v);    // quad_perm(2,3,0,1)
  v += dpp_d<0x124>(v);   // row_ror:4
  v += dpp_d<0x128>(v);   // row_ror:8
  return v;
}

// Sum over the 64 lanes of a wave, the same value (and the same rounding) in
// every lane: quad swaps and row rotations give every lane its 16-lane row
// sum, then the four row sums are added in a fixed order.
__device__ inline double wave_sum(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm(1,0,3,2)
  v += dpp_d<0x4E>(v);    // quad_perm(2,3,0,1)
  v += dpp_d<0x124>(v);   // row_ror:4
  v += dpp_d<0x128>(v);   // row_ror:8
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

}  // namespace tto
