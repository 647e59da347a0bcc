// FP64 SVD of the small R factor of each left-to-right truncation step of
// TT-round, with the truncation-rank decision made on the device.
//
// One-sided (Hestenes) Jacobi: the columns of A are rotated pairwise until
// every pair is orthogonal to relative precision.  For a square R (tall
// unfolding) A = R; its final columns are U Sigma, and W = Sigma_t V_t^T is
// formed afterwards as U_t^T R, so no rotations are accumulated.  For a wide
// R (fewer rows than columns) A = R^T, whose final columns are V Sigma, and
// the rotations are accumulated in J = U (small: k x k with k <= rows of R).
// Pairs follow the round-robin (circle) schedule in closed form, so the pairs
// of one round are disjoint and run on different waves; one workgroup
// barrier per round.
//
// Deflation: columns of A whose squared norms add up to at most
// tau^2 = (2 sqrt(nc) u ||A||_F)^2 (u = unit round-off of the arithmetic that
// produced R) are set aside before the sweeps; they change A by less than the
// rounding noise already in R.  Their energy is still counted in the
// discarded tail.  When the remaining problem fits, A and J live in LDS.
//
// Rank: the smallest t >= 1 whose discarded tail sqrt(sum_{i>t} sigma_i^2) is
// <= eps = delta/sqrt(d-1) * ||x|| (tail accumulated from the smallest
// singular value), capped by max_rank.
#include "common.h"
#include "mfma.h"
#include "wave.h"

namespace tto {

namespace {

constexpr int NT = 1024;
constexpr int NW = NT / 64;
constexpr int MAXC = SVD_SMALL_MAX;
constexpr int LDS_DOUBLES = 18000;
#ifndef JGL
#define JGL 16
#endif   // 140.6 KiB for A and J (plus ~16 KiB static)

__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}

// Pair `pair` of round `round` of the circle schedule on kp (even) players:
// player kp-1 stays, the others rotate.
__device__ inline void rr_pair(int round, int pair, int kp, int& p, int& q) {
  const int m = kp - 1;
  if (pair == 0) {
    p = m;
    q = round;
  } else {
    // round, pair < m: one conditional subtraction each instead of a remainder
    p = round + pair;
    if (p >= m) p -= m;
    q = round - pair;
    if (q < 0) q += m;
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

extern __shared__ __align__(16) double svd_lds[];

// Sum over each GL-lane group of a wave (GL = 8 or 16; every lane gets its group's sum).
template <int GL>
__device__ inline double group_sum(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm(1,0,3,2)
  v += dpp_d<0x4E>(v);    // quad_perm(2,3,0,1)
  if (GL == 8) {
    v += dpp_d<0x141>(v);   // row_half_mirror: the other quad of the 8-lane half
  } else {
    v += dpp_d<0x124>(v);   // row_ror:4
    v += dpp_d<0x128>(v);   // row_ror:8
  }
  return v;
}

// One Newton step towards 1/x from r, and towards 1/sqrt(x) from y (each
// step doubles the number of correct bits of the hardware estimate).
__device__ inline double rcp_step(double x, double r) {
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ inline double rsq_step(double x, double y) {
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// Rotation (c, s) that makes columns p and q orthogonal, from their squared
// norms al, be and their dot product ga != 0: t = tan(theta) is the root of
// smaller magnitude of t^2 + 2 zeta t - 1 = 0, zeta = (be - al) / (2 ga),
// written as t = sign(be - al) 2ga / (|be - al| + sqrt((be - al)^2 + 4ga^2))
// so that it takes one square root and one reciprocal (hardware estimates
// refined by two Newton steps); c = 1/sqrt(1 + t^2), s = c t.  Outside the
// range where the squares are safe, the quotient form is used.
__device__ inline void rotation(double al, double be, double ga, double& c, double& s) {
  const double d = be - al, g = 2.0 * ga;
  const double m = fmax(fabs(d), fabs(g));
  double t;
  if (m > 1e-150 && m < 1e150) {
    const double w = fma(d, d, g * g);
    double y = __builtin_amdgcn_rsq(w);
    y = rsq_step(w, rsq_step(w, y));
    const double den = fma(w, y, fabs(d));
    double r = __builtin_amdgcn_rcp(den);
    r = rcp_step(den, rcp_step(den, r));
    t = (d >= 0.0 ? g : -g) * r;
  } else {
    const double zeta = d / g;
    if (fabs(zeta) > 1e150) t = 0.5 / zeta;
    else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  }
  const double u = fma(t, t, 1.0);
  double cc = __builtin_amdgcn_rsq(u);
  cc = rsq_step(u, rsq_step(u, cc));
  c = cc;
  s = cc * t;
}

// One-sided Jacobi on A (len x k, column-major, leading dimension lda >= len,
// rows len..lda-1 zero); when J is requested the rotations are accumulated
// into J (k x k, column-major).
// SH: A (and J right after it) live in the dynamic LDS block, so the
// accesses compile to LDS instructions; otherwise Ag / Jg in global memory.
// A group of GL lanes handles one pair; EPL > 0 (lda == GL * EPL) keeps the
// pair's two columns in registers between the dot products and the rotation.
// rots[0] / rots[1] (shared): a rotation / a rotation with cosine above
// sqrt(tol) took place in the current sweep.  Returns the number of sweeps used.
template <bool SH, int GL, int EPL>
__device__ __attribute__((always_inline)) int jacobi(double* Ag, double* Jg, bool with_j, int len, int lda,
                                                     int k, int* rots) {
  double* A = SH ? svd_lds : Ag;
  double* J = with_j ? (SH ? svd_lds + (int64_t)lda * k : Jg) : nullptr;
  // a GL-lane group of a wave handles one pair: reductions stay inside the group
  const int tid = threadIdx.x, gl = tid % GL, grp = tid / GL;
  constexpr int NG = NT / GL;
  constexpr int NE = EPL > 0 ? EPL : 1;
  const int kp = k + (k & 1);
  const double tol = (double)len * 1.1102230246251565e-16;
  const double tol2 = tol * tol;
  int sweep = 0;
  for (; sweep < 64 && kp >= 2; ++sweep) {
    if (tid == 0) {
      rots[0] = 0;
      rots[1] = 0;
    }
    __syncthreads();
    for (int round = 0; round < kp - 1; ++round) {
      for (int pb = 0; pb < kp / 2; pb += NG) {   // uniform trip count: every group takes part in the sums
        const int pair = pb + grp;
        int p = 0, q = 0;
        if (pair < kp / 2) rr_pair(round, pair, kp, p, q);
        const bool live = pair < kp / 2 && q < k;
        if (!live) p = q = 0;
        double* ap = A + (int64_t)p * lda;
        double* aq = A + (int64_t)q * lda;
        double al = 0.0, be = 0.0, ga = 0.0;
        double x[NE], y[NE];
        if (EPL > 0) {
          // every group loads (idle groups read column 0 and drop the result)
#pragma unroll
          for (int t = 0; t < NE; ++t) {
            x[t] = ap[gl + GL * t];
            y[t] = aq[gl + GL * t];
          }
#pragma unroll
          for (int t = 0; t < NE; ++t) {
            al += x[t] * x[t];
            be += y[t] * y[t];
            ga += x[t] * y[t];
          }
        } else if (live) {
          for (int i = gl; i < len; i += GL) {
            const double u = ap[i], v = aq[i];
            al += u * u;
            be += v * v;
            ga += u * v;
          }
        }
        al = group_sum<GL>(al);
        be = group_sum<GL>(be);
        ga = group_sum<GL>(ga);
        // rotate unless the pair is orthogonal to relative precision tol
        if (live && ga != 0.0 && ga * ga > tol2 * al * be) {
          double c, s;
          rotation(al, be, ga, c, s);
          if (EPL > 0) {
#pragma unroll
            for (int e = 0; e < NE; ++e) {
              ap[gl + GL * e] = c * x[e] - s * y[e];
              aq[gl + GL * e] = s * x[e] + c * y[e];
            }
          } else {
            for (int i = gl; i < len; i += GL) {
              const double u = ap[i], v = aq[i];
              ap[i] = c * u - s * v;
              aq[i] = s * u + c * v;
            }
          }
          if (J) {
            double* jp = J + (int64_t)p * k;
            double* jq = J + (int64_t)q * k;
            for (int i = gl; i < k; i += GL) {
              const double u = jp[i], v = jq[i];
              jp[i] = c * u - s * v;
              jq[i] = s * u + c * v;
            }
          }
          if (gl == 0) {
            rots[0] = 1;
            if (ga * ga > tol * al * be) rots[1] = 1;   // a cosine above sqrt(tol)
          }
        }
      }
      __syncthreads();
    }
    const int r = rots[0], rbig = rots[1];
    __syncthreads();
    // no rotation, or only rotations with cosines below sqrt(tol): cyclic Jacobi converges
    // quadratically, so every pair is now orthogonal to about tol and a further sweep would
    // only confirm it
    if (r == 0 || rbig == 0) break;
  }
  return sweep;
}

// The sweeps of jacobi() on A in LDS (lda == GL * EPL) run by one wave alone,
// for k <= 2 * 64 / GL: one GL-lane group per pair of a round.  The LDS
// operations of one wave take effect in the order they are issued, so the
// rounds need no workgroup barrier; the other waves wait at one barrier after
// the sweeps.  Same rotations and stopping rule as jacobi().
template <int GL, int EPL>
__device__ __attribute__((always_inline)) int jacobi_wave(bool with_j, int len, int lda, int k) {
  double* A = svd_lds;
  double* J = with_j ? svd_lds + (int64_t)lda * k : nullptr;
  const int lane = threadIdx.x & 63, gl = lane % GL, grp = lane / GL;
  const int kp = k + (k & 1);
  const double tol = (double)len * 1.1102230246251565e-16;
  const double tol2 = tol * tol;
  int sweep = 0;
  for (; sweep < 64 && kp >= 2; ++sweep) {
    bool rotated = false, big = false;
    for (int round = 0; round < kp - 1; ++round) {
      int p = 0, q = 0;
      if (grp < kp / 2) rr_pair(round, grp, kp, p, q);
      const bool live = grp < kp / 2 && q < k;
      double* ap = A + (int64_t)p * lda;
      double* aq = A + (int64_t)q * lda;
      double x[EPL], y[EPL];
      if (live) {
#pragma unroll
        for (int t = 0; t < EPL; ++t) {
          x[t] = ap[gl + GL * t];
          y[t] = aq[gl + GL * t];
        }
      } else {
#pragma unroll
        for (int t = 0; t < EPL; ++t) x[t] = y[t] = 0.0;
      }
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int t = 0; t < EPL; ++t) {
        al += x[t] * x[t];
        be += y[t] * y[t];
        ga += x[t] * y[t];
      }
      al = group_sum<GL>(al);
      be = group_sum<GL>(be);
      ga = group_sum<GL>(ga);
      if (live && ga != 0.0 && ga * ga > tol2 * al * be) {
        double c, s;
        rotation(al, be, ga, c, s);
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          ap[gl + GL * e] = c * x[e] - s * y[e];
          aq[gl + GL * e] = s * x[e] + c * y[e];
        }
        if (J) {
          double* jp = J + (int64_t)p * k;
          double* jq = J + (int64_t)q * k;
          for (int i = gl; i < k; i += GL) {
            const double u = jp[i], v = jq[i];
            jp[i] = c * u - s * v;
            jq[i] = s * u + c * v;
          }
        }
        rotated = true;
        if (ga * ga > tol * al * be) big = true;
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (__ballot(rotated) == 0 || __ballot(big) == 0) break;
  }
  return sweep;
}

__global__ __launch_bounds__(NT) void k_svd(const SvdTask* __restrict__ tasks) {
  __shared__ int perm[MAXC + 2];
  __shared__ int act[MAXC];
  __shared__ double nrm2[MAXC];
  __shared__ double red[NW];
  __shared__ int rots[2], kact, lenact, tsel;
  __shared__ int wcount[NW], wmax[NW];
  __shared__ double edrop;

  const SvdTask tk = tasks[blockIdx.x];
  if (tk.block) return;   // block Jacobi (launch_svd_big)
  const int kr = tk.kr, N = tk.ncol;
  const bool tall = (kr == N);
  const int nc = kr;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // element (i, j) of A = (R or R^T); R entries below the diagonal read as zero when upper
  auto aval = [&](int i, int j) -> double {
    const int rr = tall ? i : j, cc = tall ? j : i;
    if (tk.upper && cc < rr) return 0.0;
    const int64_t e = (int64_t)rr * tk.r_ld + cc;
    return tk.r_f32 ? (double)((const float*)tk.R)[e] : ((const double*)tk.R)[e];
  };

  // ---- column norms and deflation
  if (tall) {
    // A = R (row-major): one thread per column and RG row groups, so that the reads of a
    // row are coalesced; partial sums in the LDS block (free until A is filled)
    constexpr int RG = NT / 256;
    double* part = svd_lds;
    for (int j0 = 0; j0 < nc; j0 += 256) {
      const int j = j0 + (tid & 255), g = tid >> 8;
      double s = 0.0;
      if (j < nc) {
        const int imax = (tk.upper && j + 1 < N) ? j + 1 : N;   // R(i, j) = 0 below the diagonal
        for (int i = g; i < imax; i += RG) {
          const double v = aval(i, j);
          s += v * v;
        }
      }
      part[g * 256 + (tid & 255)] = s;
      __syncthreads();
      if (g == 0 && j < nc) {
        double a = 0.0;
        for (int q = 0; q < RG; ++q) a += part[q * 256 + tid];
        nrm2[j] = a;
      }
      __syncthreads();
    }
  } else {
    // A = R^T: column j of A is row j of R (contiguous), one wave per column
    for (int j = wave; j < nc; j += NW) {
      double s = 0.0;
      for (int i = lane; i < N; i += 64) {
        const double v = aval(i, j);
        s += v * v;
      }
      s = wave_sum(s);
      if (lane == 0) nrm2[j] = s;
    }
    __syncthreads();
  }
  double tot = 0.0;
  for (int j = tid; j < nc; j += NT) tot += nrm2[j];
  tot = block_sum(tot, red);
  const double tau = 2.0 * sqrt((double)nc) * tk.bulk_u;
  const double tau2 = tau * tau * tot;
  // a column is set aside when it and every smaller column (ties by index) fit in tau^2 together
  for (int j = tid; j < nc; j += NT) {
    const double v = nrm2[j];
    double b[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // eight independent partial sums
    for (int i0 = 0; i0 < nc; i0 += 8) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = i0 + q;
        const double w = nrm2[i < nc ? i : 0];
        if (i < nc && (w < v || (w == v && i <= j))) b[q] += w;
      }
    }
    const double below = ((b[0] + b[1]) + (b[2] + b[3])) + ((b[4] + b[5]) + (b[6] + b[7]));
    perm[j] = ((below <= tau2 && tau2 > 0.0) || v == 0.0) ? 0 : 1;
  }
  __syncthreads();
  // active columns in increasing order (ballot prefix counts), the largest active index and
  // the energy set aside (nc <= MAXC = NT: one column per thread)
  {
    const bool on = tid < nc && perm[tid] != 0;
    const unsigned long long bal = __ballot(on);
    const int below_in_wave = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) {
      wcount[wave] = __popcll(bal);
      wmax[wave] = bal ? 64 * wave + 63 - __clzll(bal) : -1;   // largest active column of the wave
    }
    const double dropped = block_sum((tid < nc && !on) ? nrm2[tid] : 0.0, red);   // (contains barriers)
    int off = 0;
    for (int w = 0; w < wave; ++w) off += wcount[w];
    if (on) act[off + below_in_wave] = tid;
    if (tid == 0) {
      int k = 0, mx = -1;
      for (int w = 0; w < NW; ++w) {
        k += wcount[w];
        mx = wmax[w] > mx ? wmax[w] : mx;
      }
      kact = k;
      edrop = dropped;
      lenact = (tall && tk.upper) ? (mx + 1) : N;
    }
  }
  __syncthreads();
  const int k = kact, len = lenact > 0 ? lenact : 1;

  // ---- A_active (len x k, leading dimension lda, zero rows below len) and,
  // for a wide R, J (k x k): LDS when they fit, else global scratch.  In LDS
  // the columns are padded to a register-tile length when that fits.
  const int64_t jsz = tall ? 0 : (int64_t)k * k;
  const int epl = len <= 4 * JGL ? 4 : len <= 8 * JGL ? 8 : len <= 16 * JGL ? 16 : 0;
  int mode = -1, lda = len;   // -1: global scratch; 0: LDS, plain loops; > 0: LDS, registers
  if (epl > 0 && (int64_t)epl * JGL * k + jsz <= LDS_DOUBLES) {
    mode = epl;
    lda = epl * JGL;
  } else if ((int64_t)len * k + jsz <= LDS_DOUBLES) {
    mode = 0;
  }
  const bool in_lds = mode >= 0;
  double* A = in_lds ? svd_lds : tk.A;
  double* J = tall ? nullptr : (in_lds ? svd_lds + (int64_t)lda * k : tk.acc);
  // (the Jacobi sweeps are called with the LDS or the global pointer written
  // out, so that each copy uses LDS or global instructions, not flat ones)
  for (int64_t idx = tid; idx < (int64_t)k * lda; idx += NT) {
    const int a = (int)(idx / lda), i = (int)(idx - (int64_t)a * lda);
    A[idx] = i < len ? aval(i, act[a]) : 0.0;
  }
  for (int64_t idx = tid; idx < jsz; idx += NT) {
    const int j = (int)(idx / k), i = (int)(idx - (int64_t)j * k);
    J[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  int sweeps = 0;
  // one wave alone when every pair of a round fits in it with groups of 16 or 8 lanes
  // (narrower groups lengthen each lane's chain more than the barriers save)
  const int wgl = mode <= 0 ? 0 : (k <= 8 ? 16 : k <= 16 ? 8 : 0);
  const int wepl = wgl > 0 ? lda / wgl : 0;
  const bool one_wave = wgl > 0 && wepl <= 16;
  if (k > 0 && one_wave) {
    if (wave == 0) {
      if (wgl == 16 && wepl == 4) sweeps = jacobi_wave<16, 4>(!tall, len, lda, k);
      else if (wgl == 16 && wepl == 8) sweeps = jacobi_wave<16, 8>(!tall, len, lda, k);
      else if (wgl == 16) sweeps = jacobi_wave<16, 16>(!tall, len, lda, k);
      else if (wgl == 8 && wepl == 8) sweeps = jacobi_wave<8, 8>(!tall, len, lda, k);
      else sweeps = jacobi_wave<8, 16>(!tall, len, lda, k);
    }
    __syncthreads();
  } else if (k > 0) {
    if (mode < 0) sweeps = jacobi<false, JGL, 0>(tk.A, tk.acc, !tall, len, lda, k, rots);
    else if (mode == 4) sweeps = jacobi<true, JGL, 4>(nullptr, nullptr, !tall, len, lda, k, rots);
    else if (mode == 8) sweeps = jacobi<true, JGL, 8>(nullptr, nullptr, !tall, len, lda, k, rots);
    else if (mode == 16) sweeps = jacobi<true, JGL, 16>(nullptr, nullptr, !tall, len, lda, k, rots);
    else sweeps = jacobi<true, JGL, 0>(nullptr, nullptr, !tall, len, lda, k, rots);
  }

  // ---- singular values, order, rank
  for (int j = wave; j < k; j += NW) {
    const double* aj = A + (int64_t)j * lda;
    double s = 0.0;
    for (int i = lane; i < len; i += 64) s += aj[i] * aj[i];
    s = wave_sum(s);
    if (lane == 0) nrm2[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < k; j += NT) {
    const double sj = nrm2[j];
    int rk = 0;
    for (int i = 0; i < k; ++i) {
      const double si = nrm2[i];
      rk += (si > sj) || (si == sj && i < j);
    }
    perm[rk] = j;
    tk.sigma[rk] = sj;
  }
  __syncthreads();
  for (int i = k + tid; i < nc; i += NT) tk.sigma[i] = 0.0;
  if (tid == 0) {
    const double eps = (tk.delta_scaled > tk.eps_floor ? tk.delta_scaled : tk.eps_floor) * (*tk.norm);
    const double eps2 = eps * eps;
    int t = k > 0 ? k : 1;
    double tail = edrop;
    for (int i = k - 1; i >= 1; --i) {
      tail += tk.sigma[i] * tk.sigma[i];
      if (tail <= eps2) t = i;
      else break;
    }
    if (tk.max_rank > 0 && t > tk.max_rank) t = (int)tk.max_rank;
    if (t < 1) t = 1;
    if (k == 0 || tk.sigma[0] == 0.0) t = 1;
    tsel = t;
    *tk.rank_out = t;
    if (tk.info) *tk.info = sweeps;
  }
  __syncthreads();
  const int t = tsel;
  // position of each original column in the active list (-1 when set aside)
  for (int j = tid; j < nc; j += NT) nrm2[j] = -1.0;
  __syncthreads();
  for (int a = tid; a < k; a += NT) nrm2[act[a]] = (double)a;
  __syncthreads();
  const bool degenerate = (k == 0);
  // rows [0, len) of a square R staged in LDS beside A when they fit (W^T reads each of them t times)
  double* Rs = nullptr;
  if (tall && in_lds && (int64_t)lda * k + (int64_t)len * N <= LDS_DOUBLES) {
    Rs = svd_lds + (int64_t)lda * k;
    for (int idx = tid; idx < len * N; idx += NT) {
      const int row = idx / N, col = idx - row * N;
      Rs[idx] = aval(row, col);
    }
    __syncthreads();
  }
  // W^T: ncol x t (x ld columns, zero beyond t, when a rank bound sets the layout)
  const int ld = tk.t_ld > 0 ? tk.t_ld : t;
  for (int64_t idx = tid; idx < (int64_t)N * ld; idx += NT) {
    const int col = (int)(idx / ld), i = (int)(idx - (int64_t)col * ld);
    double v = 0.0;
    if (!degenerate && i < k && i < t) {
      const int j = perm[i];
      if (tall) {
        // row i of W = Sigma_t V_t^T = U_t^T R, with U_t = (final column)/sigma
        const double s = tk.sigma[i];
        if (s > 0.0) {
          const double* aj = A + (int64_t)j * lda;
          const int rmax = (tk.upper && col + 1 < len) ? col + 1 : len;   // R(row, col) = 0 below the diagonal
          double acc = 0.0;
          if (Rs) {
            double a4[4] = {0.0, 0.0, 0.0, 0.0};   // four independent partial sums
            for (int r0 = 0; r0 < rmax; r0 += 4) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int row = r0 + q < rmax ? r0 + q : 0;
                const double term = aj[row] * Rs[row * N + col];
                a4[q] += (r0 + q < rmax) ? term : 0.0;
              }
            }
            acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
          } else {
            for (int row = 0; row < rmax; ++row) acc += aj[row] * aval(row, col);
          }
          v = acc / s;
        }
      } else {
        v = (col < len) ? A[(int64_t)j * lda + col] : 0.0;
      }
    }
    tk.wt[idx] = v;
  }
  // U_R: kr x t (x ld columns, zero beyond t)
  for (int64_t idx = tid; idx < (int64_t)kr * ld; idx += NT) {
    const int row = (int)(idx / ld), i = (int)(idx - (int64_t)row * ld);
    double v;
    if (i >= t) {
      v = 0.0;
    } else if (degenerate || i >= k) {
      v = (row == i) ? 1.0 : 0.0;
    } else {
      const int j = perm[i];
      if (tall) {
        const double s = tk.sigma[i];
        if (s > 0.0) v = (row < len) ? A[(int64_t)j * lda + row] / s : 0.0;
        else v = (row == i) ? 1.0 : 0.0;
      } else {
        const int a = (int)nrm2[row];
        v = (a >= 0) ? J[(int64_t)j * k + a] : 0.0;
      }
    }
    tk.ur[idx] = v;
  }
}

// ---------------------------------------------------------------------------
// R factors with the block flag (more than SVD_SMALL_MAX rows, or above a
// context's crossover): block one-sided Jacobi over many workgroups, always on
// A = R^T (N x kr, column j = row j of R) with the rotations accumulated in J
// (kr x kr).  Rows of R at the noise level -- the trailing rows of the R factor
// of a matrix of low numerical rank -- are set aside first by the rule of the
// one-workgroup kernel (their energy counts in the discarded tail), so a
// low-rank R costs as little as its rank.  The active columns are split into
// blocks of BB; in each round of the circle schedule on the blocks every
// disjoint pair of blocks is one workgroup, which forms the Gram matrix G of
// its 2 BB columns on the FP64 matrix cores, reduces its off-diagonal by at
// most INNER_SWEEPS sweeps of cyclic (two-sided) Jacobi in LDS and rotates
// the columns of A and J by the accumulated rotation V.  A pair whose columns
// are orthogonal to relative precision N u is left alone; a sweep in which no
// pair needed a rotation ends the iteration (later rounds see the per-sweep
// counter and return at once).  Singular values, order, rank and the factors
// W^T (the final columns of A) and U_R (columns of J) follow.
//
// iscr layout (2 kr + 128 ints): [0, kr) order of the singular values;
// [kr, kr + 64) per-sweep rotation counters; kr + 64 rank; kr + 65 active
// count; kr + 66, kr + 67 energy set aside (a double); [kr + 128, 2 kr + 128)
// active columns in increasing order.
// ---------------------------------------------------------------------------
#ifndef BSVD_SWEEPS
#define BSVD_SWEEPS 64
#endif
#ifndef BSVD_INNER
#define BSVD_INNER 2
#endif
constexpr int BIG_SWEEPS = BSVD_SWEEPS;     // outer sweeps at most
constexpr int INNER_SWEEPS = BSVD_INNER;    // inner sweeps per pair at most
static_assert(BIG_SWEEPS <= 64, "per-sweep counters: 64 slots");
constexpr int BB = 32;              // columns per block
constexpr int PW = 2 * BB;          // columns of a pair
constexpr int GLD = PW + 1;         // padded leading dimension of G, V and the row chunk
constexpr size_t BIG_LDS = (size_t)3 * PW * GLD * 8;

struct BigSlots {
  int* order;
  int* rot;
  int* rank;
  int* kact;
  int* act;
};

__device__ inline BigSlots big_slots(const SvdTask& tk) {
  BigSlots b;
  const int k = tk.kr;
  b.order = tk.iscr;
  b.rot = tk.iscr + k;
  b.rank = tk.iscr + k + 64;
  b.kact = tk.iscr + k + 65;
  b.act = tk.iscr + k + 128;   // (kr + 66, kr + 67: the energy set aside, as the two halves of a double)
  return b;
}

// R(i, j) with the upper-triangular mask
__device__ inline double rval(const SvdTask& tk, int i, int j) {
  if (tk.upper && j < i) return 0.0;
  const int64_t e = (int64_t)i * tk.r_ld + j;
  return tk.r_f32 ? (double)((const float*)tk.R)[e] : ((const double*)tk.R)[e];
}

// A = R^T (N x kr, column-major), J = I (kr x kr), sweep counters zeroed.
__global__ __launch_bounds__(NT) void k_bsvd_prep(const SvdTask* __restrict__ tasks) {
  const SvdTask tk = tasks[blockIdx.x];
  if (!tk.block) return;
  const int N = tk.ncol, k = tk.kr;
  const int64_t stride = (int64_t)gridDim.y * NT;
  for (int64_t idx = blockIdx.y * (int64_t)NT + threadIdx.x; idx < (int64_t)N * k; idx += stride) {
    const int j = (int)(idx / N), i = (int)(idx - (int64_t)j * N);
    tk.A[idx] = rval(tk, j, i);
  }
  for (int64_t idx = blockIdx.y * (int64_t)NT + threadIdx.x; idx < (int64_t)k * k; idx += stride) {
    const int j = (int)(idx / k), i = (int)(idx - (int64_t)j * k);
    tk.acc[idx] = (i == j) ? 1.0 : 0.0;
  }
  if (blockIdx.y == 0) {
    const BigSlots b = big_slots(tk);
    for (int i = threadIdx.x; i < 64; i += NT) b.rot[i] = 0;
  }
}

// Column norms of A, the columns set aside (the largest set of smallest columns whose
// energy together is at most (2 sqrt(kr) u ||A||_F)^2, and zero columns), the active list.
__global__ __launch_bounds__(NT) void k_bsvd_deflate(const SvdTask* __restrict__ tasks) {
  __shared__ double nrm2[SVD_BIG_MAX];
  __shared__ unsigned char on[SVD_BIG_MAX];
  __shared__ double red[NW];
  const SvdTask tk = tasks[blockIdx.x];
  if (!tk.block) return;
  const int N = tk.ncol, k = tk.kr;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = wave; j < k; j += NW) {
    const double* aj = tk.A + (int64_t)j * N;
    double s0 = 0.0, s1 = 0.0;
    int i = lane;
    for (; i + 64 < N; i += 128) {
      s0 += aj[i] * aj[i];
      s1 += aj[i + 64] * aj[i + 64];
    }
    if (i < N) s0 += aj[i] * aj[i];
    const double s = wave_sum(s0 + s1);
    if (lane == 0) nrm2[j] = s;
  }
  __syncthreads();
  double tot = 0.0;
  for (int j = tid; j < k; j += NT) tot += nrm2[j];
  tot = block_sum(tot, red);
  const double tau = 2.0 * sqrt((double)k) * tk.bulk_u;
  const double tau2 = tau * tau * tot;
  for (int j = tid; j < k; j += NT) {
    const double v = nrm2[j];
    double b[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i0 = 0; i0 < k; i0 += 8) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = i0 + q;
        const double w = nrm2[i < k ? i : 0];
        if (i < k && (w < v || (w == v && i <= j))) b[q] += w;
      }
    }
    const double below = ((b[0] + b[1]) + (b[2] + b[3])) + ((b[4] + b[5]) + (b[6] + b[7]));
    on[j] = ((below <= tau2 && tau2 > 0.0) || v == 0.0) ? 0 : 1;
  }
  __syncthreads();
  if (tid == 0) {
    const BigSlots bs = big_slots(tk);
    int c = 0;
    double dropped = 0.0;
    for (int j = 0; j < k; ++j) {
      if (on[j]) bs.act[c++] = j;
      else dropped += nrm2[j];
    }
    *bs.kact = c;
    const unsigned long long bits = __double_as_longlong(dropped);
    tk.iscr[k + 66] = (int)(bits & 0xffffffffull);
    tk.iscr[k + 67] = (int)(bits >> 32);
  }
}

// Active column c (0 .. PW-1) of the pair (bp, bq): its index in A, or -1 past the last one.
__device__ inline int pair_col(int c, int bp, int bq, int kact, const int* __restrict__ act) {
  const int a = (c < BB) ? bp * BB + c : bq * BB + (c - BB);
  return a < kact ? act[a] : -1;
}

// Rows [0, rows) of the pair's columns of X (column-major, ld) times V, in place,
// 64 rows at a time through the LDS chunk.
__device__ void rotate_rows(double* __restrict__ X, int64_t ld, int rows, const int* __restrict__ cidx,
                            const double* __restrict__ V, double* __restrict__ Ch) {
  typedef Mma<double> M;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rt = wave >> 2, ct = wave & 3;
  for (int r0 = 0; r0 < rows; r0 += PW) {
    __syncthreads();
    for (int e = tid; e < PW * PW; e += NT) {
      const int c = e / PW, r = e - c * PW;
      const int j = cidx[c];
      Ch[c * GLD + r] = (j >= 0 && r0 + r < rows) ? X[(int64_t)j * ld + r0 + r] : 0.0;
    }
    __syncthreads();
    M::acc_t acc = M::zero();
#pragma unroll 4
    for (int k0 = 0; k0 < PW; k0 += 4) {
      const double a = Ch[(k0 + (lane >> 4)) * GLD + rt * 16 + (lane & 15)];   // chunk[row][k]
      const double b = V[(k0 + (lane >> 4)) * GLD + ct * 16 + (lane & 15)];    // V[k][col]
      acc = M::mma(a, b, acc);
    }
    const int c = ct * 16 + (lane & 15), j = cidx[c];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + rt * 16 + M::row(lane, v);
      if (j >= 0 && r < rows) X[(int64_t)j * ld + r] = acc[v];
    }
  }
}

__global__ __launch_bounds__(NT) void k_bsvd_round(const SvdTask* __restrict__ tasks, int sweep, int round) {
  typedef Mma<double> M;
  extern __shared__ __align__(16) double blds[];
  __shared__ int cidx[PW];
  __shared__ int pq[PW / 2][2];
  __shared__ double cs[PW / 2][2];
  __shared__ int need, inner_rot;
  const SvdTask tk = tasks[blockIdx.x];
  if (!tk.block) return;
  const BigSlots bs = big_slots(tk);
  if (sweep > 0 && bs.rot[sweep - 1] == 0) return;   // converged
  const int N = tk.ncol, k = tk.kr, kact = *bs.kact;
  const int nb = (kact + BB - 1) / BB, nbp = nb + (nb & 1);
  const int pair = blockIdx.y;
  if (nb < 2 && sweep > 0) return;   // one block: its first round orthogonalised it
  if (pair >= (nbp > 0 ? nbp / 2 : 0) || round >= (nbp > 1 ? nbp - 1 : 1)) return;
  int bp, bq;
  if (nbp >= 2) {
    rr_pair(round, pair, nbp, bp, bq);
  } else {
    bp = 0;
    bq = 1;   // a single block (at most BB active columns) with the empty one
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* G = blds;                  // PW x GLD
  double* V = blds + PW * GLD;       // PW x GLD
  double* Ch = blds + 2 * PW * GLD;  // PW x GLD
  if (tid < PW) cidx[tid] = pair_col(tid, bp, bq, kact, bs.act);
  if (tid == 0) need = 0;
  __syncthreads();
  // ---- G = A_pair^T A_pair: wave w owns the 16 x 16 tile (w / 4, w % 4)
  {
    const int ti = wave >> 2, tj = wave & 3;
    const int ja = cidx[ti * 16 + (lane & 15)], jb = cidx[tj * 16 + (lane & 15)];
    const double* Aa = tk.A + (int64_t)(ja >= 0 ? ja : 0) * N;
    const double* Ab = tk.A + (int64_t)(jb >= 0 ? jb : 0) * N;
    M::acc_t a0 = M::zero(), a1 = M::zero();
    int r0 = 0;
    for (; r0 + 8 <= N; r0 += 8) {
      const int r = r0 + (lane >> 4);
      const double x0 = ja >= 0 ? Aa[r] : 0.0, y0 = jb >= 0 ? Ab[r] : 0.0;
      const double x1 = ja >= 0 ? Aa[r + 4] : 0.0, y1 = jb >= 0 ? Ab[r + 4] : 0.0;
      a0 = M::mma(x0, y0, a0);
      a1 = M::mma(x1, y1, a1);
    }
    for (; r0 < N; r0 += 4) {
      const int r = r0 + (lane >> 4);
      const bool ok = r < N;
      const double x = (ok && ja >= 0) ? Aa[r] : 0.0, y = (ok && jb >= 0) ? Ab[r] : 0.0;
      a0 = M::mma(x, y, a0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) G[(ti * 16 + M::row(lane, v)) * GLD + tj * 16 + (lane & 15)] = a0[v] + a1[v];
  }
  __syncthreads();
  const double tol = (double)N * 1.1102230246251565e-16;
  const double tol2 = tol * tol;
  for (int e = tid; e < PW * PW; e += NT) {
    const int i = e / PW, j = e - i * PW;
    if (i < j) {
      const double ga = G[i * GLD + j], al = G[i * GLD + i], be = G[j * GLD + j];
      if (ga != 0.0 && ga * ga > tol2 * al * be) need = 1;
    }
  }
  __syncthreads();
  if (!need) return;   // the whole workgroup: no barrier is reached
  // (with the inner sweeps capped, convergence is not quadratic: a sweep ends the
  // iteration only when no pair needed any rotation)
  if (tid == 0) atomicAdd(&bs.rot[sweep], 1);
  for (int e = tid; e < PW * PW; e += NT) {
    const int i = e / PW, j = e - i * PW;
    V[i * GLD + j] = (i == j) ? 1.0 : 0.0;
  }
  // ---- cyclic Jacobi on G: rounds of PW/2 disjoint pairs, G <- J^T G J, V <- V J; a lone
  // block (the whole active set) is diagonalised to convergence, since no later round comes
  const int isw_max = (nb < 2) ? 40 : INNER_SWEEPS;
  for (int isw = 0; isw < isw_max; ++isw) {
    if (tid == 0) inner_rot = 0;
    __syncthreads();
    for (int rr = 0; rr < PW - 1; ++rr) {
      if (tid < PW / 2) {
        int p, q;
        rr_pair(rr, tid, PW, p, q);
        pq[tid][0] = p;
        pq[tid][1] = q;
        const double al = G[p * GLD + p], be = G[q * GLD + q], ga = G[p * GLD + q];
        double c = 1.0, sn = 0.0;
        if (ga != 0.0 && ga * ga > tol2 * al * be) {
          rotation(al, be, ga, c, sn);
          inner_rot = 1;
        }
        cs[tid][0] = c;
        cs[tid][1] = sn;
      }
      __syncthreads();
      for (int e = tid; e < (PW / 2) * PW; e += NT) {   // rows p, q of G
        const int pi = e / PW, j = e - pi * PW;
        const double c = cs[pi][0], sn = cs[pi][1];
        if (sn != 0.0) {
          const int p = pq[pi][0], q = pq[pi][1];
          const double u = G[p * GLD + j], w = G[q * GLD + j];
          G[p * GLD + j] = c * u - sn * w;
          G[q * GLD + j] = sn * u + c * w;
        }
      }
      __syncthreads();
      for (int e = tid; e < (PW / 2) * PW; e += NT) {   // columns p, q of G and V
        const int pi = e / PW, j = e - pi * PW;
        const double c = cs[pi][0], sn = cs[pi][1];
        if (sn != 0.0) {
          const int p = pq[pi][0], q = pq[pi][1];
          const double u = G[j * GLD + p], w = G[j * GLD + q];
          G[j * GLD + p] = c * u - sn * w;
          G[j * GLD + q] = sn * u + c * w;
          const double vu = V[j * GLD + p], vw = V[j * GLD + q];
          V[j * GLD + p] = c * vu - sn * vw;
          V[j * GLD + q] = sn * vu + c * vw;
        }
      }
      __syncthreads();
    }
    const int any = inner_rot;
    __syncthreads();   // every wave has read the flag before thread 0 clears it for the next sweep
    if (!any) break;
  }
  // ---- the pair's columns of A and of J rotated by V
  rotate_rows(tk.A, N, N, cidx, V, Ch);
  rotate_rows(tk.acc, k, k, cidx, V, Ch);
}

// Singular values (norms of the active columns), their order and the rank.
__global__ __launch_bounds__(NT) void k_bsvd_rank(const SvdTask* __restrict__ tasks) {
  __shared__ double nrm[SVD_BIG_MAX];
  const SvdTask tk = tasks[blockIdx.x];
  if (!tk.block) return;
  const BigSlots bs = big_slots(tk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = tk.ncol, k = tk.kr, kact = *bs.kact;
  for (int a = wave; a < kact; a += NW) {
    const double* aj = tk.A + (int64_t)bs.act[a] * N;
    double s0 = 0.0, s1 = 0.0;
    int i = lane;
    for (; i + 64 < N; i += 128) {
      s0 += aj[i] * aj[i];
      s1 += aj[i + 64] * aj[i + 64];
    }
    if (i < N) s0 += aj[i] * aj[i];
    const double s = wave_sum(s0 + s1);
    if (lane == 0) nrm[a] = sqrt(s);
  }
  __syncthreads();
  for (int a = tid; a < kact; a += NT) {
    const double sa = nrm[a];
    int rk = 0;
    for (int i = 0; i < kact; ++i) {
      const double si = nrm[i];
      rk += (si > sa) || (si == sa && i < a);
    }
    bs.order[rk] = bs.act[a];
    tk.sigma[rk] = sa;
  }
  __syncthreads();
  for (int i = kact + tid; i < k; i += NT) tk.sigma[i] = 0.0;
  if (tid == 0) {
    const unsigned long long bits =
        ((unsigned long long)(unsigned)tk.iscr[k + 67] << 32) | (unsigned long long)(unsigned)tk.iscr[k + 66];
    const double edrop = __longlong_as_double((long long)bits);
    const double eps = (tk.delta_scaled > tk.eps_floor ? tk.delta_scaled : tk.eps_floor) * (*tk.norm);
    const double eps2 = eps * eps;
    int t = kact > 0 ? kact : 1;
    double tail = edrop;
    for (int i = kact - 1; i >= 1; --i) {
      tail += tk.sigma[i] * tk.sigma[i];
      if (tail <= eps2) t = i;
      else break;
    }
    if (tk.max_rank > 0 && t > tk.max_rank) t = (int)tk.max_rank;
    if (t < 1) t = 1;
    if (kact == 0 || tk.sigma[0] == 0.0) t = 1;
    *tk.rank_out = t;
    *bs.rank = t;
    if (tk.info) {
      int sw = 0;
      while (sw < BIG_SWEEPS && bs.rot[sw] != 0) ++sw;
      *tk.info = sw + 1;
    }
  }
}

// W^T (N x ld): the ordered final columns of A (= V Sigma); U_R (kr x ld): the ordered
// columns of J (= U); zero beyond the rank t.  No active column (R = 0): W = 0, U_R = I_t.
__global__ __launch_bounds__(NT) void k_bsvd_copy(const SvdTask* __restrict__ tasks) {
  const SvdTask tk = tasks[blockIdx.x];
  if (!tk.block) return;
  const BigSlots bs = big_slots(tk);
  const int N = tk.ncol, k = tk.kr, kact = *bs.kact;
  const int t = *bs.rank;
  const int ld = tk.t_ld > 0 ? tk.t_ld : t;
  const int64_t stride = (int64_t)gridDim.y * NT;
  for (int64_t idx = blockIdx.y * (int64_t)NT + threadIdx.x; idx < (int64_t)k * ld; idx += stride) {
    const int row = (int)(idx / ld), i = (int)(idx - (int64_t)row * ld);
    double v = 0.0;
    if (i < t) v = (i < kact) ? tk.acc[(int64_t)bs.order[i] * k + row] : ((row == i) ? 1.0 : 0.0);
    tk.ur[idx] = v;
  }
  for (int64_t idx = blockIdx.y * (int64_t)NT + threadIdx.x; idx < (int64_t)N * ld; idx += stride) {
    const int col = (int)(idx / ld), i = (int)(idx - (int64_t)col * ld);
    tk.wt[idx] = (i < t && i < kact) ? tk.A[(int64_t)bs.order[i] * N + col] : 0.0;
  }
}

}  // namespace

hipError_t launch_svd(const SvdTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  static bool ready = false;
  if (!ready) {
    hipError_t e = hipFuncSetAttribute((const void*)k_svd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       LDS_DOUBLES * 8);
    if (e != hipSuccess) return e;
    ready = true;
  }
  hipLaunchKernelGGL(k_svd, dim3(ntasks), dim3(NT), LDS_DOUBLES * 8, s, d_tasks);
  return hipGetLastError();
}

hipError_t launch_svd_big(const SvdTask* d_tasks, int ntasks, int max_kr, hipStream_t s) {
  if (ntasks <= 0 || max_kr <= 0) return hipSuccess;
  if (max_kr > SVD_BIG_MAX) return hipErrorInvalidValue;
  static bool ready = false;
  if (!ready) {
    hipError_t e = hipFuncSetAttribute((const void*)k_bsvd_round, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)BIG_LDS);
    if (e != hipSuccess) return e;
    ready = true;
  }
  hipLaunchKernelGGL(k_bsvd_prep, dim3(ntasks, 64), dim3(NT), 0, s, d_tasks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bsvd_deflate, dim3(ntasks), dim3(NT), 0, s, d_tasks);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nb = (max_kr + BB - 1) / BB, nbp = nb + (nb & 1);
  for (int sw = 0; sw < BIG_SWEEPS; ++sw)
    for (int r = 0; r < (nbp > 1 ? nbp - 1 : 1); ++r) {
      hipLaunchKernelGGL(k_bsvd_round, dim3(ntasks, nbp > 1 ? nbp / 2 : 1), dim3(NT), BIG_LDS, s, d_tasks, sw, r);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  hipLaunchKernelGGL(k_bsvd_rank, dim3(ntasks), dim3(NT), 0, s, d_tasks);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bsvd_copy, dim3(ntasks, 64), dim3(NT), 0, s, d_tasks);
  return hipGetLastError();
}

}  // namespace tto
