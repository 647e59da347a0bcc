// Batched block-aware contraction of the right-to-left sweep of TT-round:
// core k-1 of each sum component times the transposed R factor of core k,
//   C[r][c] = sum_parts coef_p * sum_k A_p[r][k] * B[c][b_off_p + k].
// The zero blocks of the summed (block-diagonal) core are never touched:
// each component is its own part.  64x64 output tiles, 16-deep K slices
// staged in LDS, 4x4 register blocking per thread.
#include "common.h"

namespace tto {

namespace {

constexpr int TM = 64, TN = 64, TK = 16, NT = 256;

template <typename T>
__global__ __launch_bounds__(NT) void k_gemm(const GemmTask* __restrict__ tasks,
                                             const GemmPart* __restrict__ parts) {
  const GemmTask tk = tasks[blockIdx.z];
  const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
  if (row0 >= tk.M || col0 >= tk.N) return;
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (T)0;
  for (int p = 0; p < tk.nparts; ++p) {
    const GemmPart pt = parts[tk.part0 + p];
    const T* A = (const T*)pt.A;
    const T coef = (T)pt.coef;
    const int K = pt.K;
    for (int k0 = 0; k0 < K; k0 += TK) {
      for (int e = threadIdx.x; e < TM * TK; e += NT) {
        const int r = e / TK, kk = e % TK;
        const int gr = row0 + r, gk = k0 + kk;
        As[kk][r] = (gr < tk.M && gk < K) ? A[(int64_t)gr * K + gk] * coef : (T)0;
      }
      for (int e = threadIdx.x; e < TN * TK; e += NT) {
        const int c = e / TK, kk = e % TK;
        const int gc = col0 + c, gk = k0 + kk;
        T bv = (T)0;
        if (gc < tk.N && gk < K && pt.b_off + gk >= gc) {
          const int64_t bi = (int64_t)gc * tk.b_ld + pt.b_off + gk;
          bv = tk.b_f32 ? (T)((const float*)tk.B)[bi] : (T)((const double*)tk.B)[bi];
        }
        Bs[kk][c] = bv;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < TK; ++kk) {
        T a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = As[kk][tr * 4 + i];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc * 4 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
      }
      __syncthreads();
    }
  }
  T* C = (T*)tk.C;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = row0 + tr * 4 + i;
    if (r >= tk.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + tc * 4 + j;
      if (c < tk.N) C[(int64_t)r * tk.c_ld + c] = acc[i][j];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_gemm_strided(const GemmSTask* __restrict__ tasks) {
  const GemmSTask tk = tasks[blockIdx.z];
  const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
  if (row0 >= tk.M || col0 >= tk.N) return;
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  const T* A = (const T*)tk.A;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (T)0;
  for (int k0 = 0; k0 < tk.K; k0 += TK) {
    for (int e = threadIdx.x; e < TM * TK; e += NT) {
      const int r = e / TK, kk = e % TK;
      const int gr = row0 + r, gk = k0 + kk;
      As[kk][r] = (gr < tk.M && gk < tk.K) ? A[(int64_t)gr * tk.a_rs + (int64_t)gk * tk.a_cs] : (T)0;
    }
    for (int e = threadIdx.x; e < TN * TK; e += NT) {
      const int c = e / TK, kk = e % TK;
      const int gc = col0 + c, gk = k0 + kk;
      Bs[kk][c] = (gc < tk.N && gk < tk.K) ? (T)tk.B[(int64_t)gk * tk.b_rs + (int64_t)gc * tk.b_cs] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
  T* C = (T*)tk.C;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = row0 + tr * 4 + i;
    if (r >= tk.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + tc * 4 + j;
      if (c < tk.N) C[(int64_t)r * tk.c_rs + (int64_t)c * tk.c_cs] = acc[i][j];
    }
  }
}

__global__ void k_eye(double* __restrict__ X, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    X[i] = (i / n == i % n) ? 1.0 : 0.0;
}

}  // namespace

hipError_t launch_gemm_strided(int dtype, const GemmSTask* d_tasks, int ntasks, int max_m, int max_n, hipStream_t s) {
  if (ntasks <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  for (int first = 0; first < ntasks; first += 65535) {
    const int cnt = (ntasks - first) < 65535 ? (ntasks - first) : 65535;
    dim3 grid((max_n + TN - 1) / TN, (max_m + TM - 1) / TM, cnt);
    if (dtype == 0) hipLaunchKernelGGL(k_gemm_strided<double>, grid, dim3(NT), 0, s, d_tasks + first);
    else hipLaunchKernelGGL(k_gemm_strided<float>, grid, dim3(NT), 0, s, d_tasks + first);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_eye(double* X, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t total = (int64_t)n * n;
  const int blocks = (int)((total + 255) / 256 < 1024 ? (total + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_eye, dim3(blocks), dim3(256), 0, s, X, n);
  return hipGetLastError();
}

hipError_t launch_gemm(int dtype, const GemmTask* d_tasks, const GemmPart* d_parts, int ntasks, int max_m,
                       int max_n, hipStream_t s) {
  if (ntasks <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  for (int first = 0; first < ntasks; first += 65535) {
    const int cnt = (ntasks - first) < 65535 ? (ntasks - first) : 65535;
    dim3 grid((max_n + TN - 1) / TN, (max_m + TM - 1) / TM, cnt);
    if (dtype == 0) hipLaunchKernelGGL(k_gemm<double>, grid, dim3(NT), 0, s, d_tasks + first, d_parts);
    else hipLaunchKernelGGL(k_gemm<float>, grid, dim3(NT), 0, s, d_tasks + first, d_parts);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tto
