// Householder QR of tall-skinny tiles (TSQR leaves and tree nodes) and the
// application of their orthogonal factors.  These implement the QR steps of
// the right-to-left orthogonalisation sweep of TT-round and the QR that
// precedes each small SVD of the left-to-right truncation sweep.
//
// One workgroup owns one tile.  The tile lives in global memory (row-major);
// panels of QR_NB columns are factored in LDS (column-major there, so the
// per-column reductions read contiguous LDS), the per-panel blocked-WY factor
// T is formed in LDS, and the trailing columns are updated with
//   A <- A - V T^T (V^T A)
// by a 2-D thread split (columns x row groups) whose partial V^T A sums are
// combined through LDS.
//
// A tree node stacks the upper-triangular R factors of its children.  Row i
// of a stacked triangle is zero left of column i, so the Householder vectors
// of the panel starting at column p0 only touch, in each child block, the
// rows i < p0 + QR_NB: every panel works on that compacted row list only.
#include "common.h"

namespace tto {

namespace {

constexpr int NB = QR_NB;
constexpr int NT = QR_THREADS;
constexpr int MAXR = QR_MAXROWS;

__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Active tile rows of the panel [p0, p0 + nb) in increasing order; returns the count.
// Dense tile (nchild == 0): rows p0..m-1.  Node: in child block b (offset
// b*kc0, size kc_b) the local rows i with max(0, p0 - off_b) <= i < min(kc_b, p0 + nb).
__device__ int panel_rows(int* rowl, int* cnt, int m, int nchild, int kc0, int kc_last, int p0, int nb) {
  const int tid = threadIdx.x;
  if (nchild == 0) {
    for (int r = tid; r < m - p0; r += NT) rowl[r] = p0 + r;
    __syncthreads();
    return m - p0;
  }
  if (tid == 0) {
    int c = 0;
    for (int b = 0; b < nchild; ++b) {
      const int off = b * kc0;
      const int kcb = (b == nchild - 1) ? kc_last : kc0;
      const int lo = (p0 - off) > 0 ? (p0 - off) : 0;
      const int hi = kcb < (p0 + nb) ? kcb : (p0 + nb);
      for (int i = lo; i < hi; ++i) rowl[c++] = off + i;
    }
    *cnt = c;
  }
  __syncthreads();
  const int c = *cnt;
  __syncthreads();
  return c;
}

// A rows rowl[0..rows) x columns c0..c0+ncols (row-major, leading dimension lda)
//   <- A - V op(T) (V^T A),  op(T) = T^T when TRANS.
// V: LDS column-major [NB][ldv] over the compacted rows (explicit unit
// diagonal, zeros above; columns >= nb are zero); T: LDS NB x NB.
// wred: LDS scratch of NT * NB doubles.
template <bool TRANS, typename TA, typename TV>
__device__ void block_reflect(TA* __restrict__ A, int64_t lda, const int* __restrict__ rowl, int c0, int ncols,
                              int rows, const TV* __restrict__ V, int ldv, const double* __restrict__ T,
                              double* __restrict__ wred) {
  const int tid = threadIdx.x;
  const int tc = ncols < NT ? ncols : NT;
  if (tc <= 0) return;
  const int G = NT / tc;
  for (int cb = 0; cb < ncols; cb += tc) {
    const int cl = tid % tc;
    const int g = tid / tc;
    const int c = cb + cl;
    const bool active = (g < G) && (c < ncols);
    double w[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) w[k] = 0.0;
    if (active) {
      TA* col = A + (c0 + c);
      int r = g;
      for (; r + 3 * G < rows; r += 4 * G) {
        const double a0 = (double)col[(int64_t)rowl[r] * lda];
        const double a1 = (double)col[(int64_t)rowl[r + G] * lda];
        const double a2 = (double)col[(int64_t)rowl[r + 2 * G] * lda];
        const double a3 = (double)col[(int64_t)rowl[r + 3 * G] * lda];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const TV* vk = V + k * ldv;
          w[k] += (double)vk[r] * a0 + (double)vk[r + G] * a1 + (double)vk[r + 2 * G] * a2 +
                  (double)vk[r + 3 * G] * a3;
        }
      }
      for (; r < rows; r += G) {
        const double a = (double)col[(int64_t)rowl[r] * lda];
#pragma unroll
        for (int k = 0; k < NB; ++k) w[k] += (double)V[k * ldv + r] * a;
      }
    }
    double* slot = wred + (size_t)(g * tc + cl) * NB;
    if (G > 1) {
      if (g < G) {
#pragma unroll
        for (int k = 0; k < NB; ++k) slot[k] = w[k];
      }
      __syncthreads();
      if (active) {
#pragma unroll
        for (int k = 0; k < NB; ++k) w[k] = 0.0;
#pragma unroll 1
        for (int gg = 0; gg < G; ++gg) {
#pragma unroll
          for (int k = 0; k < NB; ++k) w[k] += wred[(gg * tc + cl) * NB + k];
        }
      }
      __syncthreads();
    }
    if (active) {
      // w2 = op(T) w, one output at a time through the thread's LDS slot
#pragma unroll 1
      for (int i = 0; i < NB; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NB; ++k) s += (TRANS ? T[k * NB + i] : T[i * NB + k]) * w[k];
        slot[i] = s;
      }
      double w2[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) w2[k] = slot[k];
      TA* col = A + (c0 + c);
      int r = g;
      for (; r + 3 * G < rows; r += 4 * G) {
        const int64_t i0 = (int64_t)rowl[r] * lda, i1 = (int64_t)rowl[r + G] * lda;
        const int64_t i2 = (int64_t)rowl[r + 2 * G] * lda, i3 = (int64_t)rowl[r + 3 * G] * lda;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const TV* vk = V + k * ldv;
          s0 += (double)vk[r] * w2[k];
          s1 += (double)vk[r + G] * w2[k];
          s2 += (double)vk[r + 2 * G] * w2[k];
          s3 += (double)vk[r + 3 * G] * w2[k];
        }
        const double a0 = (double)col[i0], a1 = (double)col[i1], a2 = (double)col[i2], a3 = (double)col[i3];
        col[i0] = (TA)(a0 - s0);
        col[i1] = (TA)(a1 - s1);
        col[i2] = (TA)(a2 - s2);
        col[i3] = (TA)(a3 - s3);
      }
      for (; r < rows; r += G) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NB; ++k) s += (double)V[k * ldv + r] * w2[k];
        const int64_t ia = (int64_t)rowl[r] * lda;
        col[ia] = (TA)((double)col[ia] - s);
      }
    }
    __syncthreads();
  }
}

// Build the upper-triangular T of Q = H_0 ... H_{nb-1} = I - V T V^T
// (forward, column-wise blocked WY).  S: LDS scratch NB*NB doubles.
template <typename TV>
__device__ void form_t(const TV* __restrict__ V, int ldv, int rows, int nb, const double* __restrict__ tau,
                       double* __restrict__ T, double* __restrict__ S) {
  const int tid = threadIdx.x;
  if (tid < NB * NB) {
    const int a = tid / NB, b = tid % NB;
    double s = 0.0;
    if (a < b && b < nb) {
      for (int r = b; r < rows; ++r) s += (double)V[a * ldv + r] * (double)V[b * ldv + r];
    }
    S[tid] = s;
    T[tid] = 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < nb; ++i) {
      const double ti = tau[i];
      T[i * NB + i] = ti;
      for (int a = 0; a < i; ++a) {
        double s = 0.0;
        for (int b = a; b < i; ++b) s += T[a * NB + b] * S[b * NB + i];
        T[a * NB + i] = -ti * s;
      }
    }
  }
  __syncthreads();
}

template <typename TS, typename TT>
__global__ __launch_bounds__(NT) void k_qr_factor(const QrTask* __restrict__ tasks,
                                                  const QrTask* __restrict__ children) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int rowl[MAXR];
  __shared__ int rcnt;
  const QrTask tk = tasks[blockIdx.x];
  const int m = tk.m, N = tk.ncol, tid = threadIdx.x;
  TT* A = (TT*)tk.tile;

  // ---- fill the tile
  if (tk.nchild == 0) {
    const TS* src = (const TS*)tk.src;
    const int64_t total = (int64_t)m * N;
    for (int64_t idx = tid; idx < total; idx += NT) {
      const int r = (int)(idx / N), c = (int)(idx - (int64_t)r * N);
      A[idx] = (TT)src[r * tk.src_rs + c * tk.src_cs];
    }
  } else {
    int row0 = 0;
    for (int ci = 0; ci < tk.nchild; ++ci) {
      const QrTask ch = children[tk.child0 + ci];
      const TS* ct = (const TS*)ch.tile;
      const int kc = ch.m < N ? ch.m : N;
      const int64_t total = (int64_t)kc * N;
      for (int64_t idx = tid; idx < total; idx += NT) {
        const int r = (int)(idx / N), c = (int)(idx - (int64_t)r * N);
        A[(int64_t)(row0 + r) * N + c] = (c >= r) ? (TT)ct[idx] : (TT)0;
      }
      row0 += kc;
    }
  }
  __syncthreads();

  const int kmax = m < N ? m : N;
  const int ldp = MAXR;
  TT* P = (TT*)smem;                                               // NB * MAXR
  double* T = (double*)(smem + (((size_t)NB * ldp * sizeof(TT) + 15) & ~(size_t)15));  // NB*NB
  double* S = T + NB * NB;                                         // NB*NB
  double* red = S + NB * NB;                                       // 16
  double* taus = red + 16;                                         // NB
  double* wred = taus + NB;                                        // NT*NB

  for (int p0 = 0, pi = 0; p0 < kmax; p0 += NB, ++pi) {
    const int nb = (kmax - p0) < NB ? (kmax - p0) : NB;
    const int rows = panel_rows(rowl, &rcnt, m, tk.nchild, tk.kc0, tk.kc_last, p0, nb);
    // ---- load panel (zero-padded to NB columns)
    for (int idx = tid; idx < rows * NB; idx += NT) {
      const int r = idx / NB, jj = idx - r * NB;
      P[jj * ldp + r] = (jj < nb) ? A[(int64_t)rowl[r] * N + p0 + jj] : (TT)0;
    }
    __syncthreads();
    // ---- unblocked Householder on the panel (pivot of column jj is compact row jj)
    for (int jj = 0; jj < nb; ++jj) {
      TT* col = P + jj * ldp;
      double part = 0.0;
      for (int r = jj + 1 + tid; r < rows; r += NT) {
        const double v = (double)col[r];
        part += v * v;
      }
      const double sigma = block_sum(part, red);
      const double alpha = (double)col[jj];
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (sigma != 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      __syncthreads();
      if (sigma != 0.0) {
        for (int r = jj + 1 + tid; r < rows; r += NT) col[r] = (TT)((double)col[r] * scal);
      }
      if (tid == 0) {
        col[jj] = (TT)beta;
        taus[jj] = tau;
      }
      __syncthreads();
      {
        const int c = jj + 1 + (tid >> 4);
        const int g = tid & 15;
        double w = 0.0;
        if (c < nb) {
          const TT* pc = P + c * ldp;
          if (g == 0) w = (double)pc[jj];
          for (int r = jj + 1 + g; r < rows; r += 16) w += (double)col[r] * (double)pc[r];
        }
        for (int off = 8; off > 0; off >>= 1) w += __shfl_xor(w, off, 16);
        if (c < nb && tau != 0.0) {
          TT* pc = P + c * ldp;
          const double tw = tau * w;
          if (g == 0) pc[jj] = (TT)((double)pc[jj] - tw);
          for (int r = jj + 1 + g; r < rows; r += 16) pc[r] = (TT)((double)pc[r] - tw * (double)col[r]);
        }
      }
      __syncthreads();
    }
    // ---- write the factored panel back, keep tau
    for (int idx = tid; idx < rows * nb; idx += NT) {
      const int r = idx / nb, jj = idx - r * nb;
      A[(int64_t)rowl[r] * N + p0 + jj] = P[jj * ldp + r];
    }
    if (tid < nb) tk.tau[p0 + tid] = taus[tid];
    __syncthreads();
    // ---- explicit V (unit diagonal, zeros above)
    for (int idx = tid; idx < NB * NB; idx += NT) {
      const int jj = idx / NB, r = idx - jj * NB;
      if (r <= jj && r < rows) P[jj * ldp + r] = (r == jj && jj < nb) ? (TT)1 : (TT)0;
    }
    __syncthreads();
    form_t<TT>(P, ldp, rows, nb, taus, T, S);
    if (tid < NB * NB) ((double*)tk.tmat)[(size_t)pi * NB * NB + tid] = T[tid];
    // ---- trailing update  A <- Q_p^T A  on the panel's rows
    const int c0 = p0 + nb;
    if (c0 < N) block_reflect<true, TT, TT>(A, N, rowl, c0, N - c0, rows, P, ldp, T, wred);
    __syncthreads();
  }
}

// out = Q [X; 0] for one factored tile; Q = (I - V_0 T_0 V_0^T)(I - V_1 T_1 V_1^T) ...
template <typename TT, typename TO>
__global__ __launch_bounds__(NT) void k_qr_apply(const ApplyTask* __restrict__ tasks) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int rowl[MAXR];
  __shared__ int rcnt;
  const ApplyTask tk = tasks[blockIdx.x];
  const int m = tk.m, N = tk.ncol, t = tk.t, tid = threadIdx.x;
  const TT* tile = (const TT*)tk.tile;
  double* W = tk.work;
  const int64_t total = (int64_t)m * t;
  for (int64_t idx = tid; idx < total; idx += NT) {
    const int r = (int)(idx / t), c = (int)(idx - (int64_t)r * t);
    W[idx] = (r < tk.k_in) ? tk.x[r * tk.x_ld + c] : 0.0;
  }
  __syncthreads();
  const int ldp = MAXR;
  TT* V = (TT*)smem;
  double* T = (double*)(smem + (((size_t)NB * ldp * sizeof(TT) + 15) & ~(size_t)15));
  double* wred = T + NB * NB;
  const int np = (tk.kq + NB - 1) / NB;
  for (int pi = np - 1; pi >= 0; --pi) {
    const int p0 = pi * NB;
    const int nb = (tk.kq - p0) < NB ? (tk.kq - p0) : NB;
    const int rows = panel_rows(rowl, &rcnt, m, tk.nchild, tk.kc0, tk.kc_last, p0, nb);
    for (int idx = tid; idx < rows * NB; idx += NT) {
      const int r = idx / NB, jj = idx - r * NB;
      TT v = (TT)0;
      if (jj < nb) {
        if (r == jj) v = (TT)1;
        else if (r > jj) v = tile[(int64_t)rowl[r] * N + p0 + jj];
      }
      V[jj * ldp + r] = v;
    }
    if (tid < NB * NB) T[tid] = ((const double*)tk.tmat)[(size_t)pi * NB * NB + tid];
    __syncthreads();
    block_reflect<false, double, TT>(W, t, rowl, 0, t, rows, V, ldp, T, wred);
    __syncthreads();
  }
  if (tk.to_out) {
    TO* out = (TO*)tk.out;
    for (int64_t idx = tid; idx < total; idx += NT) {
      const int r = (int)(idx / t), c = (int)(idx - (int64_t)r * t);
      out[r * tk.out_rs + c * tk.out_cs] = (TO)W[idx];
    }
  }
}

size_t factor_smem(int elt) {
  return (((size_t)NB * MAXR * elt + 15) & ~(size_t)15) + sizeof(double) * (2 * NB * NB + 16 + NB + NT * NB);
}
size_t apply_smem(int elt) {
  return (((size_t)NB * MAXR * elt + 15) & ~(size_t)15) + sizeof(double) * (NB * NB + NT * NB);
}

template <typename K>
hipError_t raise_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

hipError_t launch_qr_factor(int dtype_src, int dtype_tile, const QrTask* d_tasks, const QrTask* d_children,
                            int ntasks, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  dim3 grid(ntasks), block(NT);
  if (dtype_tile == 0) {
    const size_t sm = factor_smem(8);
    if (dtype_src == 0) hipLaunchKernelGGL((k_qr_factor<double, double>), grid, block, sm, s, d_tasks, d_children);
    else hipLaunchKernelGGL((k_qr_factor<float, double>), grid, block, sm, s, d_tasks, d_children);
  } else {
    const size_t sm = factor_smem(4);
    hipLaunchKernelGGL((k_qr_factor<float, float>), grid, block, sm, s, d_tasks, d_children);
  }
  return hipGetLastError();
}

hipError_t launch_qr_apply(int dtype_tile, int dtype_out, const ApplyTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  dim3 grid(ntasks), block(NT);
  if (dtype_tile == 0) {
    const size_t sm = apply_smem(8);
    if (dtype_out == 0) hipLaunchKernelGGL((k_qr_apply<double, double>), grid, block, sm, s, d_tasks);
    else hipLaunchKernelGGL((k_qr_apply<double, float>), grid, block, sm, s, d_tasks);
  } else {
    const size_t sm = apply_smem(4);
    if (dtype_out == 0) hipLaunchKernelGGL((k_qr_apply<float, double>), grid, block, sm, s, d_tasks);
    else hipLaunchKernelGGL((k_qr_apply<float, float>), grid, block, sm, s, d_tasks);
  }
  return hipGetLastError();
}

hipError_t qr_kernels_init() {
  hipError_t e;
  if ((e = raise_lds(k_qr_factor<double, double>, factor_smem(8))) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_factor<float, double>, factor_smem(8))) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_factor<float, float>, factor_smem(4))) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_apply<double, double>, apply_smem(8))) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_apply<double, float>, apply_smem(8))) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_apply<float, double>, apply_smem(4))) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_apply<float, float>, apply_smem(4))) != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace tto
