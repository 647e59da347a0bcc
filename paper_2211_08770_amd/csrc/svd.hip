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
#include "wave.h"

namespace tto {

namespace {

constexpr int NT = 1024;
constexpr int NW = NT / 64;
constexpr int MAXC = 1024;
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

}  // namespace tto
