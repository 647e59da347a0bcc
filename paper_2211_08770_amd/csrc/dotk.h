// TT inner product of one pair of TT-vectors (Section 2): the left-to-right
// contraction  W_k = sum_i X_k(i)^T W_{k-1} Y_k(i),  <x, y> = W_d.
//
// Step k first forms tmp = W_{k-1} * Y_k (rx_k x (n_k ry_{k+1})), then
// W_k = L(X_k)^T * tmp (tmp viewed as (rx_k n_k) x ry_{k+1}).  Both products run
// on the FP64 16x16x4 matrix cores; FP32 cores are widened to double on load, so
// every product is exact and W, tmp and all sums are FP64 in both precisions.
// One workgroup of DOT_THREADS (four waves) per pair; the long reduction of the
// second product is split over the waves when it has fewer than four output
// tiles, and the partial tiles are added in wave order, so the result does not
// depend on timing.
//
// Geo supplies n(k), x(k) = rx_k and y(k) = ry_k.  w holds 2 * wcap doubles
// (wcap >= max_k rx_k ry_k), tmp >= max_k rx_k n_k ry_{k+1} doubles; part is the
// workgroup's LDS block for the split reductions.  Returns <x, y> (every thread).
#pragma once
#include "mfma.h"
#include "wave.h"

namespace tto {

constexpr int DOT_THREADS = 256;
constexpr int DOT_WAVES = DOT_THREADS / 64;

template <typename T>
__device__ __attribute__((always_inline)) inline double ld_d(gptr<const T> p, int64_t i) {
  return (double)p[i];
}

template <typename T, typename Geo>
__device__ double dot_pair(const Geo& g, int d, const void* xp, const void* yp, double* wp, int64_t wcap,
                           double* tmpp, double (*part)[256]) {
  typedef Mma<double> M;
  const gptr<const T> X = glb((const T*)xp);
  const gptr<const T> Y = glb((const T*)yp);
  gptr<double> W = glb(wp);
  gptr<double> Wn = W + wcap;
  const gptr<double> tmp = glb(tmpp);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  if (tid == 0) W[0] = 1.0;
  __syncthreads();
  int64_t xo = 0, yo = 0;
  for (int k = 0; k < d; ++k) {
    const int64_t n = g.n(k), a0 = g.x(k), a1 = g.x(k + 1), b0 = g.y(k), b1 = g.y(k + 1);
    const gptr<const T> Xk = X + xo;
    const gptr<const T> Yk = Y + yo;
    // tmp (a0 x nb1) = W (a0 x b0) * Yk (b0 x nb1)
    {
      const int64_t nb1 = n * b1;
      const int64_t mt = (a0 + 15) >> 4, ntl = (nb1 + 15) >> 4;
      for (int64_t t = wv; t < mt * ntl; t += DOT_WAVES) {
        const int64_t r0 = (t / ntl) << 4, c0 = (t % ntl) << 4;
        const int64_t ra = r0 + lr, cb = c0 + lr;
        const bool rok = ra < a0, cok = cb < nb1;
        M::acc_t acc = M::zero();
        for (int64_t kk = 0; kk < b0; kk += 4) {
          const int64_t kq = kk + lk;
          const bool kok = kq < b0;
          const double av = (rok && kok) ? W[ra * b0 + kq] : 0.0;
          const double bv = (cok && kok) ? ld_d<T>(Yk, kq * nb1 + cb) : 0.0;
          acc = M::mma(av, bv, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = r0 + M::row(lane, v);
          if (r < a0 && cok) tmp[r * nb1 + cb] = acc[v];
        }
      }
    }
    __syncthreads();
    // Wn (a1 x b1) = L(Xk)^T (a1 x a0 n) * tmp (a0 n x b1)
    {
      const int64_t K = a0 * n;
      const int mt = (int)((a1 + 15) >> 4), ntl = (int)((b1 + 15) >> 4), tiles = mt * ntl;
      const int ks = tiles >= DOT_WAVES ? 1 : (DOT_WAVES / tiles);
      const int64_t kchunk = ((K + 4 * ks - 1) / (4 * ks)) * 4;
      for (int u = wv; u < tiles * ks; u += DOT_WAVES) {
        const int t = u / ks, part_i = u % ks;
        const int64_t r0 = (int64_t)(t / ntl) << 4, c0 = (int64_t)(t % ntl) << 4;
        const int64_t ra = r0 + lr, cb = c0 + lr;
        const bool rok = ra < a1, cok = cb < b1;
        const int64_t klo = part_i * kchunk, khi = (klo + kchunk) < K ? (klo + kchunk) : K;
        M::acc_t acc0 = M::zero(), acc1 = M::zero();
        int64_t kk = klo;
        for (; kk + 8 <= khi; kk += 8) {
          const int64_t q0 = kk + lk, q1 = kk + 4 + lk;
          const double a0v = rok ? ld_d<T>(Xk, q0 * a1 + ra) : 0.0;
          const double b0v = cok ? tmp[q0 * b1 + cb] : 0.0;
          const double a1v = rok ? ld_d<T>(Xk, q1 * a1 + ra) : 0.0;
          const double b1v = cok ? tmp[q1 * b1 + cb] : 0.0;
          acc0 = M::mma(a0v, b0v, acc0);
          acc1 = M::mma(a1v, b1v, acc1);
        }
        for (; kk < khi; kk += 4) {
          const int64_t q = kk + lk;
          const bool kok = q < khi;
          const double av = (rok && kok) ? ld_d<T>(Xk, q * a1 + ra) : 0.0;
          const double bv = (cok && kok) ? tmp[q * b1 + cb] : 0.0;
          acc0 = M::mma(av, bv, acc0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) acc0[v] += acc1[v];
        if (ks == 1) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t r = r0 + M::row(lane, v);
            if (r < a1 && cok) Wn[r * b1 + cb] = acc0[v];
          }
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) part[wv][M::row(lane, v) * 16 + lr] = acc0[v];
        }
      }
      if (ks > 1) {
        __syncthreads();
        // tile t's partials are in waves t*ks .. t*ks + ks - 1: added in that order
        for (int e = tid; e < tiles * 256; e += DOT_THREADS) {
          const int t = e >> 8, w = e & 255;
          const int64_t r = ((int64_t)(t / ntl) << 4) + (w >> 4), c = ((int64_t)(t % ntl) << 4) + (w & 15);
          double s = part[t * ks][w];
          for (int j = 1; j < ks; ++j) s += part[t * ks + j][w];
          if (r < a1 && c < b1) Wn[r * b1 + c] = s;
        }
      }
    }
    __syncthreads();
    gptr<double> sw = W;
    W = Wn;
    Wn = sw;
    xo += a0 * n * a1;
    yo += b0 * n * b1;
  }
  return W[0];
}

}  // namespace tto
