// FP64 SVD of the small R factor of each left-to-right truncation step of
// TT-round, with the truncation-rank decision made on the device.
//
// One-sided (Hestenes) Jacobi: the columns of A are rotated pairwise until
// every pair is orthogonal to relative precision; the accumulated rotations
// are kept.  For a square R (tall unfolding) A = R and the accumulated
// rotations are V; for a wide R (fewer rows than columns) A = R^T and the
// accumulated rotations are the left singular vectors.  Pairs follow a
// round-robin tournament so that each round's pairs are disjoint and run on
// different waves.
//
// Rank: the smallest t >= 1 whose discarded tail sqrt(sum_{i>t} sigma_i^2) is
// <= eps = delta/sqrt(d-1) * ||x|| (tail accumulated from the smallest
// singular value), capped by max_rank.
#include "common.h"

namespace tto {

namespace {

constexpr int NT = 512;
constexpr int MAXC = 1024;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(NT) void k_svd(const SvdTask* __restrict__ tasks) {
  const SvdTask tk = tasks[blockIdx.x];
  const int kr = tk.kr, N = tk.ncol;
  const bool tall = (kr == N);
  const int len = N, nc = kr;
  double* A = tk.A;
  double* J = tk.acc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = NT / 64;

  __shared__ int perm[MAXC + 2];
  __shared__ double sig[MAXC];
  __shared__ int rots;
  __shared__ int tsel;

  for (int64_t idx = tid; idx < (int64_t)nc * len; idx += NT) {
    const int j = (int)(idx / len), i = (int)(idx - (int64_t)j * len);
    // an upper-trapezoidal R stores Householder vectors below its diagonal: read them as zero
    const int rr = tall ? i : j, cc = tall ? j : i;
    A[idx] = (tk.upper && cc < rr) ? 0.0 : tk.R[(int64_t)rr * tk.r_ld + cc];
  }
  for (int64_t idx = tid; idx < (int64_t)nc * nc; idx += NT) {
    const int j = (int)(idx / nc), i = (int)(idx - (int64_t)j * nc);
    J[idx] = (i == j) ? 1.0 : 0.0;
  }
  const int ncp = nc + (nc & 1);
  for (int i = tid; i < ncp; i += NT) perm[i] = i;
  __syncthreads();

  const double tol = sqrt((double)len) * 1.1102230246251565e-16;
  int sweep = 0;
  for (; sweep < 64 && ncp >= 2; ++sweep) {
    if (tid == 0) rots = 0;
    __syncthreads();
    for (int round = 0; round < ncp - 1; ++round) {
      for (int pair = wave; pair < ncp / 2; pair += nwaves) {
        int p = perm[pair], q = perm[ncp - 1 - pair];
        if (p >= nc || q >= nc) continue;
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        double* ap = A + (int64_t)p * len;
        double* aq = A + (int64_t)q * len;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < len; i += 64) {
          const double x = ap[i], y = aq[i];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga != 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
          const double zeta = (be - al) / (2.0 * ga);
          double t;
          if (fabs(zeta) > 1e150) t = 0.5 / zeta;
          else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          for (int i = lane; i < len; i += 64) {
            const double x = ap[i], y = aq[i];
            ap[i] = c * x - s * y;
            aq[i] = s * x + c * y;
          }
          double* jp = J + (int64_t)p * nc;
          double* jq = J + (int64_t)q * nc;
          for (int i = lane; i < nc; i += 64) {
            const double x = jp[i], y = jq[i];
            jp[i] = c * x - s * y;
            jq[i] = s * x + c * y;
          }
          if (lane == 0) atomicAdd(&rots, 1);
        }
      }
      __syncthreads();
      if (tid == 0 && ncp > 2) {
        const int last = perm[ncp - 1];
        for (int i = ncp - 1; i >= 2; --i) perm[i] = perm[i - 1];
        perm[1] = last;
      }
      __syncthreads();
    }
    const int r = rots;
    __syncthreads();
    if (r == 0) break;
  }

  // singular values = column norms
  for (int j = wave; j < nc; j += nwaves) {
    const double* aj = A + (int64_t)j * len;
    double s = 0.0;
    for (int i = lane; i < len; i += 64) s += aj[i] * aj[i];
    s = wave_sum(s);
    if (lane == 0) sig[j] = sqrt(s);
  }
  __syncthreads();
  // rank sort (decreasing, ties by index) -> perm[rank] = column
  for (int j = tid; j < nc; j += NT) {
    const double sj = sig[j];
    int rk = 0;
    for (int i = 0; i < nc; ++i) {
      const double si = sig[i];
      rk += (si > sj) || (si == sj && i < j);
    }
    perm[rk] = j;
    tk.sigma[rk] = sj;
  }
  __syncthreads();
  if (tid == 0) {
    const double eps = tk.delta_scaled * (*tk.norm);
    const double eps2 = eps * eps;
    int t = nc;
    double tail = 0.0;
    for (int i = nc - 1; i >= 1; --i) {
      tail += tk.sigma[i] * tk.sigma[i];
      if (tail <= eps2) t = i;
      else break;
    }
    if (tk.max_rank > 0 && t > tk.max_rank) t = (int)tk.max_rank;
    if (t < 1) t = 1;
    if (tk.sigma[0] == 0.0) t = 1;
    tsel = t;
    *tk.rank_out = t;
    if (tk.info) *tk.info = sweep;
  }
  __syncthreads();
  const int t = tsel;
  for (int64_t idx = tid; idx < (int64_t)N * t; idx += NT) {
    const int col = (int)(idx / t), i = (int)(idx - (int64_t)col * t);
    const int j = perm[i];
    tk.wt[idx] = tall ? tk.sigma[i] * J[(int64_t)j * nc + col] : A[(int64_t)j * len + col];
  }
  for (int64_t idx = tid; idx < (int64_t)kr * t; idx += NT) {
    const int row = (int)(idx / t), i = (int)(idx - (int64_t)row * t);
    const int j = perm[i];
    double v;
    if (tall) {
      const double s = tk.sigma[i];
      v = (s > 0.0) ? A[(int64_t)j * len + row] / s : (row == i ? 1.0 : 0.0);
    } else {
      v = J[(int64_t)j * nc + row];
    }
    tk.ur[idx] = v;
  }
}

}  // namespace

hipError_t launch_svd(const SvdTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_svd, dim3(ntasks), dim3(NT), 0, s, d_tasks);
  return hipGetLastError();
}

}  // namespace tto
