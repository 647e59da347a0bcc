// Small kernels of the TT hot path: TT inner products (batched over
// component pairs; the contraction itself is in dotk.h), norms and scaling,
// copies of TT-sum blocks (segments, row blocks with dtype conversion) and the
// materialised axpy, the in-place compaction of bound-planned result cores,
// the FP64 Cholesky + triangular inverse of the Gram scheme, the MGS and
// serving projection coefficients, the matrices whose 2-norms give the loss of
// orthogonality, the TT-Householder helpers (canonical basis, R column,
// reflection and q coefficients) and the Laplacian TT-matrix core product.
#include <algorithm>

#include "common.h"
#include "dotk.h"
#include "wave.h"

namespace tto {

namespace {

constexpr int NT = 256;

__device__ inline double block_sum256(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  __syncthreads();
  return s;
}

// <x, y> for one component pair: the contraction of dot_pair (dotk.h) with the
// geometry of the pair in device arrays.
struct DotGeoDev {
  const int64_t* nn;
  const int64_t* rx;
  const int64_t* ry;
  __device__ int64_t n(int k) const { return nn[k]; }
  __device__ int64_t x(int k) const { return rx[k]; }
  __device__ int64_t y(int k) const { return ry[k]; }
};

template <typename T>
__global__ __launch_bounds__(DOT_THREADS) void k_dot(const DotTask* __restrict__ tasks) {
  __shared__ double part[DOT_THREADS / 64][256];
  const DotTask tk = tasks[blockIdx.x];
  const DotGeoDev g{tk.nn, tk.rx, tk.ry};
  const double v = dot_pair<T>(g, tk.d, tk.x, tk.y, (double*)tk.w, tk.wcap, (double*)tk.tmp, part);
  if (threadIdx.x == 0) *tk.out = tk.coef * v;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_sumsq(const T* __restrict__ x, int64_t n, double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double v = (double)x[i];
    s += v * v;
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) *out = sqrt(s);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_sumsq_batched(const SumsqTask* __restrict__ tasks) {
  __shared__ double red[16];
  const SumsqTask tk = tasks[blockIdx.x];
  const gptr<const T> x = glb((const T*)tk.x);
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < tk.n; i += 1024) {
    const double v = (double)x[i];
    s += v * v;
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) *glb(tk.out) = sqrt(s);
}

template <typename T>
__global__ void k_scale(T* __restrict__ x, int64_t n, const double* __restrict__ nrm) {
  const double v = *nrm;
  const double inv = v > 0.0 ? 1.0 / v : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (T)((double)x[i] * inv);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_copy_segs(const CopySeg* __restrict__ segs) {
  const CopySeg sg = segs[blockIdx.y];
  const T* src = (const T*)sg.src;
  T* dst = (T*)sg.dst;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < sg.count; i += (int64_t)gridDim.x * NT) {
    const double v = sg.coef * (double)src[i];
    dst[i] = sg.accumulate ? (T)((double)dst[i] + v) : (T)v;
  }
}

// One row of a block per workgroup step, the threads along the row (coalesced
// on both sides).
__global__ __launch_bounds__(NT) void k_block_copy(const BlockCopy* __restrict__ tasks) {
  const BlockCopy tk = tasks[blockIdx.y];
  for (int r = blockIdx.x; r < tk.rows; r += gridDim.x) {
    const int64_t so = (int64_t)r * tk.src_ld, dof = (int64_t)r * tk.dst_ld;
    for (int c = threadIdx.x; c < tk.cols; c += NT) {
      double v = 0.0;
      if (tk.src && !(tk.tri && c < r))
        v = tk.src_f32 ? (double)((const float*)tk.src)[so + c] : ((const double*)tk.src)[so + c];
      if (tk.dst_f32) ((float*)tk.dst)[dof + c] = (float)v;
      else ((double*)tk.dst)[dof + c] = v;
    }
  }
}

__global__ void k_segsum(const double* __restrict__ slots, const int32_t* __restrict__ seg,
                         const int32_t* __restrict__ idx, int nout, double* __restrict__ out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int i = seg[o]; i < seg[o + 1]; ++i) s += slots[i];
  out[idx ? idx[o] : o] = s;
}

// In-place lower Cholesky of the row-major m x m matrix G, then
// Rinv = (L^T)^{-1} (upper triangular, row-major).  info = 0 on success,
// j+1 when the j-th pivot is <= m u G_jj (G numerically not SPD; u is the unit
// round-off of the arithmetic that formed G).
__global__ __launch_bounds__(NT) void k_cholinv(double* __restrict__ G, int m, double* __restrict__ Rinv,
                                                int32_t* __restrict__ info, double u) {
  __shared__ int fail;
  const int tid = threadIdx.x;
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    if (tid == 0) {
      const double gjj = G[j * m + j];
      double dj = gjj;
      for (int k = 0; k < j; ++k) dj -= G[j * m + k] * G[j * m + k];
      // numerically singular once the pivot falls to the rounding level of G_jj
      if (!(dj > (double)m * u * gjj)) fail = j + 1;
      else G[j * m + j] = sqrt(dj);
    }
    __syncthreads();
    if (fail) break;
    for (int i = j + 1 + tid; i < m; i += NT) {
      double s = G[i * m + j];
      for (int k = 0; k < j; ++k) s -= G[i * m + k] * G[j * m + k];
      G[i * m + j] = s / G[j * m + j];
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) *info = fail;
    return;
  }
  // R = L^T: R[r][k] = G[k*m + r].  Column c of R^{-1} by back substitution.
  for (int c = tid; c < m; c += NT) {
    for (int r = m - 1; r >= 0; --r) {
      double v = 0.0;
      if (r <= c) {
        double s = (r == c) ? 1.0 : 0.0;
        for (int k = r + 1; k <= c; ++k) s -= G[k * m + r] * Rinv[k * m + c];
        v = s / G[r * m + r];
      }
      Rinv[r * m + c] = v;
    }
  }
  if (tid == 0) *info = 0;
}

// E_k = I_k - G[:k, :k] for k = 1..m, stored back to back (row-major k x k).
// Leading k x k blocks of the m x m matrix G, packed one after another:
// E_k = I - G_k (loss of orthogonality) or E_k = G_k (condition numbers).
__global__ void k_loo_mats(const double* __restrict__ G, int m, double* __restrict__ E, int minus_identity) {
  const int k = blockIdx.x + 1;
  double* Ek = E + (int64_t)(k - 1) * k * (2 * k - 1) / 6;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int r = e / k, c = e - r * k;
    Ek[e] = minus_identity ? (r == c ? 1.0 : 0.0) - G[r * m + c] : G[r * m + c];
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_axpy(const AxpyTask* __restrict__ tasks) {
  const AxpyTask tk = tasks[blockIdx.y];
  const int zr0 = tk.first ? 1 : tk.xr0 + tk.yr0;
  const int zr1 = tk.last ? 1 : tk.xr1 + tk.yr1;
  const int64_t total = (int64_t)zr0 * tk.n * zr1;
  const T* X = (const T*)tk.x;
  const T* Y = (const T*)tk.y;
  T* Z = (T*)tk.z;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int a = (int)(e / ((int64_t)tk.n * zr1));
    const int64_t rem = e - (int64_t)a * tk.n * zr1;
    const int i = (int)(rem / zr1), b = (int)(rem - (int64_t)i * zr1);
    double v = 0.0;
    const bool inx = (tk.first || a < tk.xr0) && (tk.last || b < tk.xr1);
    const bool iny = (tk.first || a >= tk.xr0) && (tk.last || b >= tk.xr1);
    if (inx) {
      const int ax = tk.first ? 0 : a, bx = tk.last ? 0 : b;
      v += tk.alpha * (double)X[((int64_t)ax * tk.n + i) * tk.xr1 + bx];
    }
    if (iny) {
      const int ay = tk.first ? 0 : a - tk.xr0, by = tk.last ? 0 : b - tk.xr1;
      v += (double)Y[((int64_t)ay * tk.n + i) * tk.yr1 + by];
    }
    Z[e] = (T)v;
  }
}

__global__ void k_mgs_correct(const double* __restrict__ dots, const double* __restrict__ Gq, int ldg, int i,
                              double* __restrict__ r, double* __restrict__ neg) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int j = 0; j < i; ++j) {
    double s = dots[j];
    for (int l = 0; l < j; ++l) s -= r[l] * Gq[(int64_t)l * ldg + j];
    r[j] = s;
    if (neg) neg[j] = -s;
  }
}

__global__ void k_coef_batched(const CoefTask* __restrict__ tasks, int ntasks) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntasks) return;
  const CoefTask tk = tasks[t];
  for (int j = 0; j < tk.b; ++j) {
    double s = tk.dots[j];
    if (tk.modified && tk.gram)
      for (int l = 0; l < j; ++l) s -= tk.r[l] * tk.gram[(int64_t)l * tk.b + j];
    tk.r[j] = s;
  }
}

// Canonical basis TT-vectors e_{first}, ..., e_{first+count-1} (0-based linear
// indices; Section 3.3): rank-one cores holding a one at i_k of the multi-index
// phi(i), first index varying fastest, zero elsewhere.  Vector v is stored at
// out[v*S, v*S + S) with S = sum_k n_k, core k at offset sum_{l<k} n_l.
template <typename T>
__global__ void k_canonical(T* __restrict__ out, const int64_t* __restrict__ nn, int d, int64_t S, int64_t first,
                            int count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * count) return;
  const int64_t v = e / S, pos = e - v * S;
  int64_t rest = first + v, off = 0;
  T val = (T)0;
  for (int k = 0; k < d; ++k) {
    const int64_t n = nn[k];
    const int64_t ik = rest % n;
    rest /= n;
    if (pos < off + n) {
      val = (pos - off == ik) ? (T)1 : (T)0;
      break;
    }
    off += n;
  }
  out[e] = val;
}

// Column i of R and the coefficients of the Householder sum (Algorithm 6) from
// dots[j] = <a, e_j> (j <= i) and dots[i+1] = <a, a> (or ||a|| when norm_given):  R(j, i) = dots[j] for
// j < i; R(i, i) = -s sqrt(<a, a> - sum_{j<i} dots[j]^2) with s = +1 when
// dots[i] > 0 and -1 otherwise (the stable sign); coef[j] = -R(j, i), j <= i.
// A remainder that is not positive (a in the span of e_0..e_{i-1}) gives
// R(i, i) = 0, which the host reports as a breakdown.
__global__ void k_hh_column(const double* __restrict__ dots, int i, int norm_given, double* __restrict__ Rcol,
                            double* __restrict__ coef) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int j = 0; j < i; ++j) {
    const double r = dots[j];
    Rcol[j] = r;
    coef[j] = -r;
    s = s + r * r;
  }
  const double aa = norm_given ? dots[i + 1] * dots[i + 1] : dots[i + 1];
  const double g2 = aa - s;
  const double sign = dots[i] > 0.0 ? 1.0 : -1.0;
  const double rii = g2 > 0.0 ? -sign * sqrt(g2) : 0.0;
  Rcol[i] = rii;
  coef[i] = -rii;
}

// Reflection of the later vectors by u_i in component form (Algorithm 8 with
// a~_j = a_j + sum_{l<i} C(j, l) u_l):  <a~_j, u_i> = <a_j, u_i> + sum_{l<i}
// C(j, l) <u_l, u_i>, and C(j, i) = -2 <a~_j, u_i> for j = i+1..m-1.
// dots_a[j-i-1] = <a_j, u_i>; G[i*m + l] = <u_l, u_i> (l < i); Ct[l*m + j] = C(j, l).
__global__ void k_hh_reflect(const double* __restrict__ dots_a, const double* __restrict__ G,
                             double* __restrict__ Ct, int m, int i) {
  const int j = i + 1 + blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double s = dots_a[j - i - 1];
  for (int l = 0; l < i; ++l) s += Ct[(int64_t)l * m + j] * G[(int64_t)i * m + l];
  Ct[(int64_t)i * m + j] = -2.0 * s;
}

// Coefficients of q_i = H_0 ... H_i e_i (Algorithm 8) in component form: the
// reflections j = i, i-1, ..., 0 in turn, <q~_i, u_j> = <e_i, u_j> +
// sum_{l=j+1..i} D(i, l) <u_l, u_j> and D(i, j) = -2 <q~_i, u_j>.
// EU[i*m + j] = <e_i, u_j> (j <= i), G[l*m + j] = <u_l, u_j> (j < l),
// D[i*m + j].  One thread per i (the recurrence runs down j).
__global__ void k_hh_qcoef(const double* __restrict__ EU, const double* __restrict__ G, double* __restrict__ D,
                           int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  for (int j = i; j >= 0; --j) {
    double s = EU[(int64_t)i * m + j];
    for (int l = j + 1; l <= i; ++l) s += D[(int64_t)i * m + l] * G[(int64_t)l * m + j];
    D[(int64_t)i * m + j] = -2.0 * s;
  }
}

// One core of y = alpha * Delta_d x (Section 4: the Dirichlet Laplacian of
// order d as the rank-two TT-matrix with cores [L, I], [[I, 0], [L, I]] and
// [I; L], L = (n+1)^2 tridiag(1, -2, 1)).  kind: 0 first core (1 x n x 2r1:
// blocks L X, X), 1 interior (2r0 x n x 2r1: blocks X, 0 / L X, X), 2 last core
// (2r0 x n x 1: blocks X / L X), 3 the only core (L X).  X row-major
// [r0][n][r1]; one thread per output element; the second difference reads the
// neighbours of mode index i (zero outside [0, n)).
template <typename T>
__global__ void k_laplacian_core(const T* __restrict__ X, int64_t r0, int64_t n, int64_t r1, int kind,
                                 double alpha, T* __restrict__ Y) {
  const int64_t R0 = (kind == 1 || kind == 2) ? 2 * r0 : r0;
  const int64_t R1 = (kind == 0 || kind == 1) ? 2 * r1 : r1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= R0 * n * R1) return;
  const int64_t A = e / (n * R1), rem = e - A * n * R1, i = rem / R1, B = rem - i * R1;
  const int ba = (A >= r0) ? 1 : 0, bb = (B >= r1) ? 1 : 0;   // block row and column
  const int64_t a = A - ba * r0, b = B - bb * r1;
  // which block: 0 zero, 1 X, 2 L X
  int blk;
  if (kind == 3) blk = 2;
  else if (kind == 0) blk = bb ? 1 : 2;
  else if (kind == 2) blk = ba ? 2 : 1;
  else blk = (ba == 0) ? (bb ? 0 : 1) : (bb ? 1 : 2);
  double v = 0.0;
  const T* xa = X + (a * n) * r1 + b;
  if (blk == 1) {
    v = (double)xa[i * r1];
  } else if (blk == 2) {
    const double s = (double)(n + 1) * (double)(n + 1);
    double t = -2.0 * (double)xa[i * r1];
    if (i > 0) t += (double)xa[(i - 1) * r1];
    if (i + 1 < n) t += (double)xa[(i + 1) * r1];
    v = s * t;
  }
  if (kind == 0 || kind == 3) v *= alpha;
  Y[e] = (T)v;
}

template <typename TS, typename TD>
__global__ void k_cast(const TS* __restrict__ x, TD* __restrict__ y, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = (TD)x[e];
}

template <typename T>
__global__ void k_fill_const(T* __restrict__ x, int64_t n, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = (T)v;
}

// Deterministic values in [-1, 1) from an integer hash of the index (synthetic
// matrices for timing tile shapes; the values do not matter to the timing).
template <typename T>
__global__ void k_fill_pattern(T* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 32;
    x[i] = (T)((double)(h >> 11) * (1.0 / 4503599627370496.0) - 1.0);
  }
}

__global__ void k_add(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

__global__ void k_neg(const double* __restrict__ a, double* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = -a[i];
}

__global__ void k_sym_lower(double* __restrict__ G, int m) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int i = e / m, j = e - i * m;
  if (j > i) G[e] = G[j * m + i];
}

__global__ void k_tril(const double* __restrict__ L, int m, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int i = e / m, j = e - i * m;
  out[e] = (j <= i) ? L[e] : 0.0;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_compact(const CompactTask* __restrict__ tasks) {
  constexpr int U = 8;   // elements per thread and chunk
  const CompactTask tk = tasks[blockIdx.x];
  const int d = tk.d;
  if (threadIdx.x == 0) {
    tk.ranks[0] = 1;
    tk.ranks[d] = 1;
    *tk.status = tk.init_status;
  }
  if (!tk.active) return;
  const int64_t* n = tk.geo;
  const int64_t* tb = tk.geo + d;
  const int64_t* so = tk.geo + 2 * d + 1;
  const gptr<const T> src = glb((const T*)tk.staging);
  const gptr<T> dst = glb((T*)tk.out);
  const bool in_place = tk.staging == tk.out;
  // every thread walks the same offsets.  Element e of core k moves from so_k + row tb_{k+1} + b
  // to off_k + row t_{k+1} + b (row = a n_k + i): never to a higher address, and in the order of
  // the sources, so a chunk is read completely before it is written and no write reaches a
  // source that is still to be read (off_k <= so_k, t <= tb).
  int64_t off = 0;
  for (int k = 0; k < d; ++k) {
    const int64_t t0 = k == 0 ? 1 : tk.ranks[k], t1 = k + 1 == d ? 1 : tk.ranks[k + 1];
    const int64_t nk = n[k], sz = t0 * nk * t1;
    if (t0 > tb[k] || t1 > tb[k + 1]) {   // a rank above its bound: never read past the core
      if (threadIdx.x == 0) *tk.status = -7;
      return;
    }
    if (off + sz > tk.capacity) {
      if (threadIdx.x == 0) *tk.status = -3;
      return;
    }
    if (!(in_place && off == so[k] && t0 == tb[k] && t1 == tb[k + 1])) {   // else already in place
      const int32_t w = (int32_t)t1, wb = (int32_t)tb[k + 1];
      for (int64_t base = 0; base < sz; base += (int64_t)U * NT) {
        T v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const int64_t e = base + j * NT + threadIdx.x;
          const int32_t row = (int32_t)(e / w), b = (int32_t)(e - (int64_t)row * w);
          v[j] = e < sz ? src[so[k] + (int64_t)row * wb + b] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const int64_t e = base + j * NT + threadIdx.x;
          if (e < sz) dst[off + e] = v[j];
        }
        __syncthreads();
      }
    }
    off += sz;
  }
}

}  // namespace

hipError_t launch_compact(int dtype, const CompactTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  if (dtype == 0) hipLaunchKernelGGL(k_compact<double>, dim3(ntasks), dim3(NT), 0, s, d_tasks);
  else hipLaunchKernelGGL(k_compact<float>, dim3(ntasks), dim3(NT), 0, s, d_tasks);
  return hipGetLastError();
}

hipError_t launch_axpy(int dtype, const AxpyTask* d_tasks, int ntasks, int64_t max_elems, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  int bx = (int)((max_elems + NT - 1) / NT);
  if (bx > 4096) bx = 4096;
  if (bx < 1) bx = 1;
  dim3 grid(bx, ntasks);
  if (dtype == 0) hipLaunchKernelGGL(k_axpy<double>, grid, dim3(NT), 0, s, d_tasks);
  else hipLaunchKernelGGL(k_axpy<float>, grid, dim3(NT), 0, s, d_tasks);
  return hipGetLastError();
}

hipError_t launch_mgs_correct(const double* dots, const double* Gq, int ldg, int i, double* r, double* neg,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_mgs_correct, dim3(1), dim3(64), 0, s, dots, Gq, ldg, i, r, neg);
  return hipGetLastError();
}

hipError_t launch_canonical(int dtype, void* out, const int64_t* d_n, int d, int64_t S, int64_t first, int count,
                            hipStream_t s) {
  const int64_t total = S * count;
  if (total <= 0) return hipSuccess;
  const int blocks = (int)((total + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_canonical<double>, dim3(blocks), dim3(256), 0, s, (double*)out, d_n, d, S, first, count);
  else
    hipLaunchKernelGGL(k_canonical<float>, dim3(blocks), dim3(256), 0, s, (float*)out, d_n, d, S, first, count);
  return hipGetLastError();
}

hipError_t launch_hh_column(const double* dots, int i, int norm_given, double* Rcol, double* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_hh_column, dim3(1), dim3(64), 0, s, dots, i, norm_given, Rcol, coef);
  return hipGetLastError();
}

hipError_t launch_laplacian_core(int dtype, const void* X, int64_t r0, int64_t n, int64_t r1, int kind, double alpha,
                                 void* Y, hipStream_t s) {
  const int64_t R0 = (kind == 1 || kind == 2) ? 2 * r0 : r0;
  const int64_t R1 = (kind == 0 || kind == 1) ? 2 * r1 : r1;
  const int64_t total = R0 * n * R1;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (dtype == 0)
    hipLaunchKernelGGL(k_laplacian_core<double>, dim3((unsigned)blocks), dim3(256), 0, s, (const double*)X, r0, n, r1,
                       kind, alpha, (double*)Y);
  else
    hipLaunchKernelGGL(k_laplacian_core<float>, dim3((unsigned)blocks), dim3(256), 0, s, (const float*)X, r0, n, r1,
                       kind, alpha, (float*)Y);
  return hipGetLastError();
}

hipError_t launch_cast(int src_dtype, const void* x, int dst_dtype, void* y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks), b(256);
  if (src_dtype == 1 && dst_dtype == 0) hipLaunchKernelGGL((k_cast<float, double>), g, b, 0, s, (const float*)x, (double*)y, n);
  else if (src_dtype == 0 && dst_dtype == 1) hipLaunchKernelGGL((k_cast<double, float>), g, b, 0, s, (const double*)x, (float*)y, n);
  else if (src_dtype == 0) hipLaunchKernelGGL((k_cast<double, double>), g, b, 0, s, (const double*)x, (double*)y, n);
  else hipLaunchKernelGGL((k_cast<float, float>), g, b, 0, s, (const float*)x, (float*)y, n);
  return hipGetLastError();
}

hipError_t launch_fill_const(int dtype, void* x, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (dtype == 0) hipLaunchKernelGGL(k_fill_const<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)x, n, v);
  else hipLaunchKernelGGL(k_fill_const<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)x, n, v);
  return hipGetLastError();
}

hipError_t launch_hh_reflect(const double* dots_a, const double* G, double* Ct, int m, int i, hipStream_t s) {
  const int n = m - 1 - i;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hh_reflect, dim3((n + 63) / 64), dim3(64), 0, s, dots_a, G, Ct, m, i);
  return hipGetLastError();
}

hipError_t launch_hh_qcoef(const double* EU, const double* G, double* D, int m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hh_qcoef, dim3((m + 63) / 64), dim3(64), 0, s, EU, G, D, m);
  return hipGetLastError();
}

hipError_t launch_coef_batched(const CoefTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coef_batched, dim3((ntasks + 63) / 64), dim3(64), 0, s, d_tasks, ntasks);
  return hipGetLastError();
}

hipError_t launch_fill_pattern(int dtype, void* x, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  if (dtype == 0) hipLaunchKernelGGL(k_fill_pattern<double>, dim3(blocks), dim3(256), 0, s, (double*)x, n);
  else hipLaunchKernelGGL(k_fill_pattern<float>, dim3(blocks), dim3(256), 0, s, (float*)x, n);
  return hipGetLastError();
}

hipError_t launch_add(const double* a, const double* b, double* out, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add, dim3((n + 255) / 256), dim3(256), 0, s, a, b, out, n);
  return hipGetLastError();
}

hipError_t launch_neg(const double* a, double* out, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_neg, dim3((n + 255) / 256), dim3(256), 0, s, a, out, n);
  return hipGetLastError();
}

hipError_t launch_sym_lower(double* G, int m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_lower, dim3((m * m + 255) / 256), dim3(256), 0, s, G, m);
  return hipGetLastError();
}

hipError_t launch_tril(const double* L, int m, double* out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tril, dim3((m * m + 255) / 256), dim3(256), 0, s, L, m, out);
  return hipGetLastError();
}

hipError_t launch_dot(int dtype, const DotTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  if (dtype == 0) hipLaunchKernelGGL(k_dot<double>, dim3(ntasks), dim3(DOT_THREADS), 0, s, d_tasks);
  else hipLaunchKernelGGL(k_dot<float>, dim3(ntasks), dim3(DOT_THREADS), 0, s, d_tasks);
  return hipGetLastError();
}

hipError_t launch_sumsq(int dtype, const void* x, int64_t n, double* out, hipStream_t s) {
  if (dtype == 0) hipLaunchKernelGGL(k_sumsq<double>, dim3(1), dim3(1024), 0, s, (const double*)x, n, out);
  else hipLaunchKernelGGL(k_sumsq<float>, dim3(1), dim3(1024), 0, s, (const float*)x, n, out);
  return hipGetLastError();
}

hipError_t launch_sumsq_batched(int dtype, const SumsqTask* d_tasks, int ntasks, hipStream_t s) {
  for (int first = 0; first < ntasks; first += 65535) {
    const int cnt = (ntasks - first) < 65535 ? (ntasks - first) : 65535;
    if (dtype == 0) hipLaunchKernelGGL(k_sumsq_batched<double>, dim3(cnt), dim3(1024), 0, s, d_tasks + first);
    else hipLaunchKernelGGL(k_sumsq_batched<float>, dim3(cnt), dim3(1024), 0, s, d_tasks + first);
  }
  return hipGetLastError();
}

hipError_t launch_scale(int dtype, void* x, int64_t n, const double* nrm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)((n + NT - 1) / NT < 1024 ? (n + NT - 1) / NT : 1024);
  if (dtype == 0) hipLaunchKernelGGL(k_scale<double>, dim3(blocks), dim3(NT), 0, s, (double*)x, n, nrm);
  else hipLaunchKernelGGL(k_scale<float>, dim3(blocks), dim3(NT), 0, s, (float*)x, n, nrm);
  return hipGetLastError();
}

hipError_t launch_copy_segs(int dtype, const CopySeg* d_segs, int nsegs, hipStream_t s) {
  for (int first = 0; first < nsegs; first += 65535) {
    const int cnt = (nsegs - first) < 65535 ? (nsegs - first) : 65535;
    dim3 grid(16, cnt);
    if (dtype == 0) hipLaunchKernelGGL(k_copy_segs<double>, grid, dim3(NT), 0, s, d_segs + first);
    else hipLaunchKernelGGL(k_copy_segs<float>, grid, dim3(NT), 0, s, d_segs + first);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_block_copy(const BlockCopy* d_tasks, int ntasks, int64_t max_rows, hipStream_t s) {
  if (ntasks <= 0 || max_rows <= 0) return hipSuccess;
  const int gx = (int)(max_rows < 512 ? max_rows : 512);
  for (int first = 0; first < ntasks; first += 65535) {
    const int cnt = (ntasks - first) < 65535 ? (ntasks - first) : 65535;
    hipLaunchKernelGGL(k_block_copy, dim3(gx, cnt), dim3(NT), 0, s, d_tasks + first);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_segsum(const double* slots, const int32_t* seg, const int32_t* idx, int nout, double* out,
                         hipStream_t s) {
  if (nout <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_segsum, dim3((nout + 255) / 256), dim3(256), 0, s, slots, seg, idx, nout, out);
  return hipGetLastError();
}

hipError_t launch_cholinv(double* G, int m, double* Rinv, int32_t* info, double u, hipStream_t s) {
  hipLaunchKernelGGL(k_cholinv, dim3(1), dim3(NT), 0, s, G, m, Rinv, info, u);
  return hipGetLastError();
}

hipError_t launch_loo_mats(const double* G, int m, double* E, int minus_identity, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_loo_mats, dim3(m), dim3(NT), 0, s, G, m, E, minus_identity);
  return hipGetLastError();
}

}  // namespace tto
