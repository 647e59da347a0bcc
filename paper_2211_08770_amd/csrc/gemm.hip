// Batched block-aware contraction of the right-to-left sweep of TT-round:
// core k-1 of each sum component times the transposed R factor of core k,
//   C[r][c] = sum_parts coef_p * sum_k A_p[r][k] * B[c][b_off_p + k],
// and the strided products C = A B of the left-to-right sweep (explicitly
// formed orthogonal factors) and of the randomized rounding.
// The zero blocks of the summed (block-diagonal) core are never touched:
// each component is its own part.  Both run on the 16x16x4 matrix cores in the
// precision of the data (FP32 MFMA with FP32 accumulation for FP32-bulk, FP64
// otherwise): a workgroup of four waves owns a 64 x 64 output tile, K is staged
// through LDS 16 at a time (k-major, so the 16 lanes of an operand read 16
// consecutive entries), and wave w computes output rows 16w..16w+15 against
// the four 16-column blocks (four accumulators, four MFMAs per K-step of 4).
#include "common.h"
#include "mfma.h"
#include "wave.h"

namespace tto {

namespace {

constexpr int TM = 64, TN = 64, TK = 16, NT = 256;

// One K-slice of 16 from the LDS stage into the four accumulators of this wave.
template <typename T>
__device__ __attribute__((always_inline)) void mma_slice(const T (*As)[TM + 1], const T (*Bs)[TN + 1],
                                                        typename Mma<T>::acc_t (&acc)[4]) {
  typedef Mma<T> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rl = lane & 15, kl = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < TK; k0 += 4) {
    const T a = As[k0 + kl][16 * wave + rl];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = M::mma(a, Bs[k0 + kl][16 * j + rl], acc[j]);
  }
}

// Stores this wave's 16 x 64 block of the tile: register v of lane l is row
// Mma::row(l, v), column l % 16 of each 16-column block.
template <typename T, typename F>
__device__ __attribute__((always_inline)) void store_tile(const typename Mma<T>::acc_t (&acc)[4], int row0, int col0,
                                                         F&& put) {
  typedef Mma<T> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) put(row0 + 16 * wave + M::row(lane, v), col0 + 16 * j + (lane & 15), acc[j][v]);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_gemm(const GemmTask* __restrict__ tasks,
                                             const GemmPart* __restrict__ parts) {
  typedef Mma<T> M;
  const GemmTask tk = tasks[blockIdx.z];
  const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
  if (row0 >= tk.M || col0 >= tk.N) return;
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  typename M::acc_t acc[4] = {M::zero(), M::zero(), M::zero(), M::zero()};
  for (int p = 0; p < tk.nparts; ++p) {
    const GemmPart pt = parts[tk.part0 + p];
    const gptr<const T> A = glb((const T*)pt.A);
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
          bv = tk.b_f32 ? (T)glb((const float*)tk.B)[bi] : (T)glb((const double*)tk.B)[bi];
        }
        Bs[kk][c] = bv;
      }
      __syncthreads();
      mma_slice<T>(As, Bs, acc);
      __syncthreads();
    }
  }
  const gptr<T> C = glb((T*)tk.C);
  store_tile<T>(acc, row0, col0, [&](int r, int c, T v) {
    if (r < tk.M && c < tk.N) C[(int64_t)r * tk.c_ld + c] = v;
  });
}

template <typename T>
__global__ __launch_bounds__(NT) void k_gemm_strided(const GemmSTask* __restrict__ tasks) {
  typedef Mma<T> M;
  const GemmSTask tk = tasks[blockIdx.z];
  const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
  if (row0 >= tk.M || col0 >= tk.N) return;
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  const gptr<const T> A = glb((const T*)tk.A);
  const gptr<const double> B = glb(tk.B);
  typename M::acc_t acc[4] = {M::zero(), M::zero(), M::zero(), M::zero()};
  for (int k0 = 0; k0 < tk.K; k0 += TK) {
    for (int e = threadIdx.x; e < TM * TK; e += NT) {
      const int r = e / TK, kk = e % TK;
      const int gr = row0 + r, gk = k0 + kk;
      As[kk][r] = (gr < tk.M && gk < tk.K) ? A[(int64_t)gr * tk.a_rs + (int64_t)gk * tk.a_cs] : (T)0;
    }
    for (int e = threadIdx.x; e < TN * TK; e += NT) {
      const int c = e / TK, kk = e % TK;
      const int gc = col0 + c, gk = k0 + kk;
      Bs[kk][c] = (gc < tk.N && gk < tk.K) ? (T)B[(int64_t)gk * tk.b_rs + (int64_t)gc * tk.b_cs] : (T)0;
    }
    __syncthreads();
    mma_slice<T>(As, Bs, acc);
    __syncthreads();
  }
  const gptr<T> C = glb((T*)tk.C);
  store_tile<T>(acc, row0, col0, [&](int r, int c, T v) {
    if (r < tk.M && c < tk.N) C[(int64_t)r * tk.c_rs + (int64_t)c * tk.c_cs] = v;
  });
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
