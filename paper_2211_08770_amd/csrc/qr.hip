// Householder QR of tall-skinny tiles (TSQR leaves and tree nodes) and the
// application of their orthogonal factors.  These implement the QR steps of
// the right-to-left orthogonalisation sweep of TT-round and the QR that
// precedes each small SVD of the left-to-right truncation sweep.
//
// One workgroup (16 waves) owns one tile held row-major in global memory.
//  * Panels of QR_NB = 16 columns: panel column c lives in the registers of
//    wave c (lane l holds rows l, l + 64, ...), in double.  For column j the
//    owner publishes the column in LDS; every wave reads it, forms the
//    reflector itself (same arithmetic, same result in every wave) and
//    reduces, in one pass over its rows, the squared norm and the dot product
//    with its own column: waves right of j update their column, waves left of
//    j (already finished) produce the entries S(c, j) of V^T V for the compact
//    WY form.  One workgroup barrier per column.
//  * The blocked update of the trailing columns uses the 16x16x4 MFMA
//    (f64 for FP64 tiles, f32 for FP32-bulk tiles) for all three products of
//    Q^T A = A - V T^T (V^T A): W = V^T A, Y = T^T W and A -= V Y, where the
//    panel's reflectors H_0 ... H_15 = I - V T V^T (T upper triangular, formed
//    from S and tau).  T is stored per panel; applying Q uses Y = T W instead.
//    When the trailing block has fewer 16-column tiles than there are waves,
//    the rows of each tile are split over several waves whose partial V^T A
//    are summed in LDS, so every wave has work.
//  * A tree node stacks the upper-triangular R factors of its children.  Row
//    i of a stacked triangle is zero left of column i, so the reflectors of
//    the panel starting at column p0 only touch, in each child block, the
//    rows i < p0 + 16: every panel works on that compacted row list.
#include "common.h"
#include "mfma.h"
#include "wave.h"

namespace tto {

namespace {

constexpr int NB = QR_NB;       // 16: panel width = MFMA tile edge
constexpr int NT = QR_THREADS;  // 1024 = 16 waves
constexpr int NWV = NT / 64;
static_assert(NWV >= QR_NB, "the panel factorisation gives every panel column its own wave");
constexpr int MAXR = QR_MAXROWS;
constexpr int XSTRIDE = ((MAXR + 63) / 64) * 64;   // a published column: every row slot of every lane
// LDS scratch after the panel: two column buffers during the panel
// factorisation, partial V^T A of row-split tiles during the update.
constexpr int SCR_DOUBLES = (2 * XSTRIDE > NWV * NB * NB) ? 2 * XSTRIDE : NWV * NB * NB;

// Active tile rows of the panel [p0, p0 + nb) in increasing order; returns the count.
// Dense tile (nchild == 0): rows p0..m-1.  Node: in child block b (offset
// b*kc0, size kc_b) the local rows i with max(0, p0 - off_b) <= i < min(kc_b, p0 + nb).
__device__ __attribute__((always_inline)) int panel_rows(int* rowl, int* bstart, int m, int nchild, int kc0, int kc_last, int p0, int nb) {
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
      bstart[b] = c;
      c += (hi > lo) ? (hi - lo) : 0;
    }
    bstart[nchild] = c;
  }
  __syncthreads();
  for (int b = 0; b < nchild; ++b) {
    const int off = b * kc0;
    const int lo = (p0 - off) > 0 ? (p0 - off) : 0;
    const int c0 = bstart[b], cnt = bstart[b + 1] - c0;
    for (int i = tid; i < cnt; i += NT) rowl[c0 + i] = off + lo + i;
  }
  const int total = bstart[nchild];
  __syncthreads();
  return total;
}

// B operand of K-step s (rows 4s..4s+3) taken from a 16x16 MFMA result in
// D layout: lane l needs D[4s + l/16][l%16].
__device__ inline double bop(const v4d& d, int s) { return d[s]; }   // f64: same lane, register s
__device__ inline float bop(const v4f& d, int s) {                 // f32: lane 16s + l%16, register l/16
  const int lane = threadIdx.x & 63;
  const int src = 16 * s + (lane & 15);
  const float t0 = __shfl(d[0], src, 64), t1 = __shfl(d[1], src, 64);
  const float t2 = __shfl(d[2], src, 64), t3 = __shfl(d[3], src, 64);
  const int q = lane >> 4;
  return q == 0 ? t0 : (q == 1 ? t1 : (q == 2 ? t2 : t3));
}

// Partial W = V^T A over the rows [rlo, rhi) (rlo a multiple of 16) of the
// 16-column tile at column `col`; four accumulators keep four MFMAs in flight.
template <typename TA, typename TV>
__device__ __attribute__((always_inline)) typename Mma<TV>::acc_t wpartial(
    gptr<const TA> __restrict__ A, int64_t lda, const int* __restrict__ rowl, int col, bool colok, int rlo, int rhi,
    const TV* __restrict__ V, int ldv) {
  typedef Mma<TV> M;
  const int lane = threadIdx.x & 63;
  typename M::acc_t w0 = M::zero(), w1 = M::zero(), w2 = M::zero(), w3 = M::zero();
  constexpr int U = 12;   // K-steps whose global loads are issued together
  // every load is issued unconditionally from a valid address (rows past rhi and
  // columns past the tile read row rlo / column 0) and masked afterwards, so the
  // row-list reads and then the global loads go out back to back
  const int colc = colok ? col : 0;
  for (int r0 = rlo; r0 < rhi; r0 += 4 * U) {
    int ri[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + 4 * u + (lane >> 4);
      ri[u] = rowl[r < rhi ? r : rlo];
    }
    TA g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) g[u] = A[(int64_t)ri[u] * lda + colc];
    TV b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + 4 * u + (lane >> 4);
      b[u] = (r < rhi && colok) ? (TV)g[u] : (TV)0;
    }
#pragma unroll
    for (int u = 0; u < U; u += 4) {
      TV a[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = r0 + 4 * u + (lane >> 4) + 4 * k;
        const TV vv = V[(lane & 15) * ldv + (r < rhi ? r : rlo)];
        a[k] = (r < rhi) ? vv : (TV)0;
      }
      w0 = M::mma(a[0], b[u], w0);
      w1 = M::mma(a[1], b[u + 1], w1);
      w2 = M::mma(a[2], b[u + 2], w2);
      w3 = M::mma(a[3], b[u + 3], w3);
    }
  }
  return (w0 + w1) + (w2 + w3);
}

// A -= V Y on the rows [rlo, rhi) (rlo a multiple of 16) of the tile's column;
// yb holds Y in B-operand layout.  The A values of UB row blocks are loaded together.
template <typename TA, typename TV>
__device__ __attribute__((always_inline)) void update_rows(gptr<TA> __restrict__ A, int64_t lda,
                                                           const int* __restrict__ rowl, int col, bool colok, int rlo,
                                                           int rhi, const TV* __restrict__ V, int ldv,
                                                           const TV (&yb)[4]) {
  typedef Mma<TV> M;
  const int lane = threadIdx.x & 63;
  constexpr int UB = 2;
  const int colc = colok ? col : 0;
  for (int rb0 = rlo; rb0 < rhi; rb0 += NB * UB) {
    // row-list reads, then the loads of the old values (valid addresses, masked later)
    int idx[UB][4];   // tile element offsets (a tile holds < 2^31 elements)
#pragma unroll
    for (int ub = 0; ub < UB; ++ub)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rb0 + NB * ub + M::row(lane, v);
        idx[ub][v] = (int)((int64_t)rowl[r < rhi ? r : rlo] * lda + colc);
      }
    TA old[UB][4];
#pragma unroll
    for (int ub = 0; ub < UB; ++ub)
#pragma unroll
      for (int v = 0; v < 4; ++v) old[ub][v] = A[idx[ub][v]];
    // every loaded value is needed in a register here: the compiler may not sink a load
    // into its conditional store below (a full round trip inside the store sequence)
#pragma unroll
    for (int ub = 0; ub < UB; ++ub)
#pragma unroll
      for (int v = 0; v < 4; ++v) asm volatile("" ::"v"(old[ub][v]));
#pragma unroll
    for (int ub = 0; ub < UB; ++ub) {
      const int ra = rb0 + NB * ub + (lane & 15);
      typename M::acc_t d = M::zero();
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const TV vv = V[(4 * s + (lane >> 4)) * ldv + (ra < rhi ? ra : rlo)];
        d = M::mma((ra < rhi) ? vv : (TV)0, yb[s], d);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rb0 + NB * ub + M::row(lane, v);
        if (colok && r < rhi) A[idx[ub][v]] = (TA)((double)old[ub][v] - (double)d[v]);
      }
    }
  }
}

// Trailing block update of the rows rowl[0..rows) x columns [c0, ncol) of A:
//   FORWARD:  A <- Q^T A = A - V T^T (V^T A)   (factorisation)
//   !FORWARD: A <- Q A   = A - V T (V^T A)     (application)
// V: LDS column-major [NB][ldv] with explicit unit diagonal and zeros above;
// Tm: LDS NB x NB row-major upper-triangular T (zero beyond the panel width);
// wpart: LDS scratch of NWV x 256 doubles.  Called by the whole workgroup.
template <bool FORWARD, typename TA, typename TV>
__device__ __attribute__((always_inline)) void block_update(gptr<TA> __restrict__ A, int64_t lda, const int* __restrict__ rowl, int c0, int ncol,
                             int rows, const TV* __restrict__ V, int ldv, const double* __restrict__ Tm,
                             double* __restrict__ wpart) {
  typedef Mma<TV> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ntile = (ncol - c0 + NB - 1) / NB;
  if (ntile <= 0 || rows <= 0) return;
  // A operand of op(T) for the 4 K-steps: op(T)[l%16][4s + l/16]
  TV ta[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = lane & 15, k = 4 * s + (lane >> 4);
    ta[s] = (TV)(FORWARD ? Tm[k * NB + i] : Tm[i * NB + k]);
  }
  int nsplit = 1;
  while (nsplit * 2 * ntile <= NWV && nsplit * 2 * NB <= rows) nsplit *= 2;
  if (nsplit == 1) {
    for (int tile = wave; tile < ntile; tile += NWV) {
      const int col = c0 + tile * NB + (lane & 15);
      const bool colok = col < ncol;
      const typename M::acc_t w = wpartial<TA, TV>(A, lda, rowl, col, colok, 0, rows, V, ldv);
      typename M::acc_t y = M::zero();
#pragma unroll
      for (int s = 0; s < 4; ++s) y = M::mma(ta[s], bop(w, s), y);
      TV yb[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) yb[s] = bop(y, s);
      update_rows<TA, TV>(A, lda, rowl, col, colok, 0, rows, V, ldv, yb);
    }
    return;
  }
  // fewer tiles than waves: nsplit waves share a tile, each on a chunk of rows
  const int tile = wave / nsplit, part = wave - tile * nsplit;
  const bool act = tile < ntile;
  const int chunk = (((rows + nsplit - 1) / nsplit) + NB - 1) & ~(NB - 1);
  const int rlo = part * chunk < rows ? part * chunk : rows;
  const int rhi = rlo + chunk < rows ? rlo + chunk : rows;
  const int col = c0 + tile * NB + (lane & 15);
  const bool colok = act && col < ncol;
  if (act) {
    const typename M::acc_t w = wpartial<TA, TV>(A, lda, rowl, col, colok, rlo, rhi, V, ldv);
#pragma unroll
    for (int v = 0; v < 4; ++v) wpart[wave * 256 + v * 64 + lane] = (double)w[v];
  }
  __syncthreads();
  if (act) {
    // every wave of the tile sums the partials in the same order: identical W
    double ws[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = 0; p < nsplit; ++p) {
#pragma unroll
      for (int v = 0; v < 4; ++v) ws[v] += wpart[(tile * nsplit + p) * 256 + v * 64 + lane];
    }
    typename M::acc_t w;
#pragma unroll
    for (int v = 0; v < 4; ++v) w[v] = (TV)ws[v];
    typename M::acc_t y = M::zero();
#pragma unroll
    for (int s = 0; s < 4; ++s) y = M::mma(ta[s], bop(w, s), y);
    TV yb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) yb[s] = bop(y, s);
    update_rows<TA, TV>(A, lda, rowl, col, colok, rlo, rhi, V, ldv, yb);
  }
}

// Publish panel column j for the next step: its entries below the diagonal
// (zeros elsewhere, up to the last used row slot) to xs, and its Householder
// reflector parameters to prm = {tau, scal, beta}: H = I - tau v v^T with
// v = [1; scal * x], beta the new diagonal.  Called by the owning wave.
template <int RT>
__device__ __attribute__((always_inline)) void publish(const double (&y)[RT], int j, int rows, int rt, double* __restrict__ xs,
                               double* __restrict__ prm) {
  const int lane = threadIdx.x & 63;
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    if (t < rt) {
      const int r = lane + 64 * t;
      const double v = (r > j && r < rows) ? y[t] : 0.0;
      xs[r] = v;
      if (t & 1) s1 += v * v;
      else s0 += v * v;
    }
  }
  const double sigma = wave_sum(s0 + s1);
  const double alpha = readlane_d(y[0], j);
  double tau = 0.0, beta = alpha, scal = 0.0;
  if (sigma != 0.0) {
    const double w = fma(alpha, alpha, sigma);
    if (w > 1e-280 && w < 1e280) {
      // hardware estimates of 1/sqrt and 1/x, each refined by two Newton steps
      double ys = __builtin_amdgcn_rsq(w);
      ys = fma(0.5 * ys, fma(-w * ys, ys, 1.0), ys);
      ys = fma(0.5 * ys, fma(-w * ys, ys, 1.0), ys);
      const double nrm = w * ys;
      beta = (alpha >= 0.0) ? -nrm : nrm;
      double rb = __builtin_amdgcn_rcp(beta);
      rb = fma(rb, fma(-beta, rb, 1.0), rb);
      rb = fma(rb, fma(-beta, rb, 1.0), rb);
      tau = (beta - alpha) * rb;
      const double den = alpha - beta;
      double rs = __builtin_amdgcn_rcp(den);
      rs = fma(rs, fma(-den, rs, 1.0), rs);
      scal = fma(rs, fma(-den, rs, 1.0), rs);
    } else {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = (alpha >= 0.0) ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
  }
  if (lane == 0) {
    prm[0] = tau;
    prm[1] = scal;
    prm[2] = beta;
  }
}

__host__ __device__ inline size_t panel_bytes(int elt, int ldv) {
  return ((size_t)NB * ldv * elt + 15) & ~(size_t)15;
}

// Strictly upper part of S = V^T V (columns >= nb zero) for the compact WY
// form.  V: LDS column-major [NB][ldv], rows [0, rows).  The rows are split
// over the waves in multiples of 4; every wave's 16x16 partial goes to part
// (NWV x 256 doubles of LDS) and thread (i, j) sums the partials in wave order.
template <typename TV>
__device__ __attribute__((always_inline)) void gram_v(const TV* __restrict__ V, int ldv, int rows, int nb, double* __restrict__ part,
                       double* __restrict__ S) {
  typedef Mma<TV> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int chunk = (((rows + NWV - 1) / NWV) + 3) & ~3;
  const int rlo = wave * chunk, rhi = (rlo + chunk < rows) ? rlo + chunk : rows;
  typename M::acc_t c0 = M::zero(), c1 = M::zero();
  int r0 = rlo;
  for (; r0 + 4 < rhi; r0 += 8) {
    const int r = r0 + (lane >> 4);
    const TV a0 = V[(lane & 15) * ldv + r];
    const TV a1 = (r + 4 < rhi) ? V[(lane & 15) * ldv + r + 4] : (TV)0;
    c0 = M::mma(a0, a0, c0);
    c1 = M::mma(a1, a1, c1);
  }
  if (r0 < rhi) {
    const int r = r0 + (lane >> 4);
    const TV a0 = (r < rhi) ? V[(lane & 15) * ldv + r] : (TV)0;
    c0 = M::mma(a0, a0, c0);
  }
  const typename M::acc_t acc = c0 + c1;
#pragma unroll
  for (int v = 0; v < 4; ++v) part[wave * 256 + M::row(lane, v) * NB + (lane & 15)] = (double)acc[v];
  __syncthreads();
  if (threadIdx.x < NB * NB) {
    const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
    double s = 0.0;
    for (int w = 0; w < NWV; ++w) s += part[w * 256 + threadIdx.x];
    S[threadIdx.x] = (i < j && j < nb) ? s : 0.0;
  }
  __syncthreads();
}

// T of the compact WY form H_0 ... H_15 = I - V T V^T (forward): T_ii = tau_i,
// and two adjacent blocks of reflectors with factors T1, T2 combine into
// [[T1, -T1 S12 T2], [0, T2]] with S12 = V1^T V2 (a block of S).  The 4 x 4
// diagonal blocks come from the recurrence T_rc = -tau_c sum_b T_rb S_bc directly; blocks of 4 and
// 8 columns are then combined in two levels, every element of a level's
// products by its own thread (two barrier-separated steps, at most 8 terms
// each).  S (LDS, strictly upper V^T V) and tau (LDS) are inputs; a zero
// tau gives a zero row and column.  Called by the whole workgroup.
__device__ __attribute__((always_inline)) void form_t(const double* __restrict__ S, const double* __restrict__ tau,
                                                      double* __restrict__ Tm) {
  __shared__ double Mt[NB * NB];
  const int tid = threadIdx.x;
  const int r = (tid >> 4) & (NB - 1), c = tid & (NB - 1);
  const bool mine = tid < NB * NB;
  // 4 x 4 diagonal blocks directly: row r of a block by the recurrence
  // T_rc = -tau_c sum_{r <= b < c} T_rb S_bc (at most three terms), each element by its own thread
  if (mine) {
    double v = 0.0;
    const int d = c - r;
    if ((c & ~3) == (r & ~3) && d >= 0) {
      const double t0 = tau[r];
      v = t0;
      if (d >= 1) {
        const double t1 = -tau[r + 1] * (t0 * S[r * NB + r + 1]);
        v = t1;
        if (d >= 2) {
          const double t2 = -tau[r + 2] * (t0 * S[r * NB + r + 2] + t1 * S[(r + 1) * NB + r + 2]);
          v = t2;
          if (d >= 3)
            v = -tau[r + 3] * (t0 * S[r * NB + r + 3] + t1 * S[(r + 1) * NB + r + 3] + t2 * S[(r + 2) * NB + r + 3]);
        }
      }
    }
    Tm[tid] = v;
  }
  __syncthreads();
#pragma unroll 1
  for (int h = 4; h < NB; h <<= 1) {
    const int p = (r / (2 * h)) * (2 * h);
    const bool in12 = mine && (c / (2 * h)) == (r / (2 * h)) && (r - p) < h && (c - p) >= h;
    if (in12) {   // M = S12 T2 (T2 upper triangular)
      double m = 0.0;
#pragma unroll 1
      for (int k = p + h; k <= c; ++k) m += S[r * NB + k] * Tm[k * NB + c];
      Mt[tid] = m;
    }
    __syncthreads();
    if (in12) {   // T12 = -T1 M (T1 upper triangular)
      double t = 0.0;
#pragma unroll 1
      for (int k = r; k < p + h; ++k) t += Tm[r * NB + k] * Mt[k * NB + c];
      Tm[tid] = -t;
    }
    __syncthreads();
  }
}

// Householder factorisation of the nb columns of one panel held in P (LDS,
// column-major [NB][ldv], rows [0, rows)): column c in the registers of wave c
// (RS row slots per lane, rows <= 64 RS); per column the owner publishes it
// (xs, prm in scr), every later column's wave takes one dot product and
// updates itself: one workgroup barrier per column.  On return P holds the
// factored panel (R on and above the diagonal, V below) and taus the tau.
template <typename TT, int RS>
__device__ __attribute__((always_inline)) void panel_columns(TT* __restrict__ P, int ldv, int rows, int nb,
                                                             double* __restrict__ scr, double* __restrict__ prm,
                                                             double* __restrict__ taus) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rt = (rows + 63) >> 6;
  const bool mine = wave < nb;
  double y[RS];
#pragma unroll
  for (int t = 0; t < RS; ++t) {
    const int r = lane + 64 * t;
    y[t] = (mine && t < rt && r < rows) ? (double)P[wave * ldv + r] : 0.0;
  }
  if (wave == 0) publish(y, 0, rows, rt, scr, prm);
  __syncthreads();
  for (int jj = 0; jj < nb; ++jj) {
    if (mine && wave >= jj) {
      // column jj below its diagonal (zero elsewhere) and its reflector
      const double* xs = scr + (jj & 1) * XSTRIDE;
      const double* pp = prm + (jj & 1) * 4;
      // all loads first (no wait between them), then the products
      double x[RS];
#pragma unroll
      for (int t = 0; t < RS; ++t) {
        // unconditional load (the buffer holds every row slot), masked value: no branch per slot
        const double v = xs[lane + 64 * t];
        x[t] = (t < rt) ? v : 0.0;
      }
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int t = 0; t < RS; ++t) {
        if (t & 1) d1 += x[t] * y[t];
        else d0 += x[t] * y[t];
      }
      const double tau = pp[0], scal = pp[1];
      if (wave > jj) {
        // apply H_jj to the own column
        const double dot = wave_sum(d0 + d1);
        if (tau != 0.0) {
          const double tw = tau * (scal * dot + readlane_d(y[0], jj));
          const double f = tw * scal;
#pragma unroll
          for (int t = 0; t < RS; ++t) y[t] -= f * x[t];
          if (lane == jj) y[0] -= tw;
        }
        if (wave == jj + 1) publish(y, jj + 1, rows, rt, scr + ((jj + 1) & 1) * XSTRIDE, prm + ((jj + 1) & 1) * 4);
      } else if (wave == jj) {
        // the own column becomes beta on the diagonal and the reflector below
        // (rounded to the tile precision: the MFMA updates use that V)
        if (tau != 0.0) {
#pragma unroll
          for (int t = 0; t < RS; ++t)
            if (t < rt && lane + 64 * t > jj) y[t] = (double)(TT)(y[t] * scal);
        }
        if (lane == jj) y[0] = pp[2];
        if (lane == 0) taus[jj] = tau;
      }
    }
    __syncthreads();
  }
  // ---- factored panel back to LDS
  if (mine) {
#pragma unroll
    for (int t = 0; t < RS; ++t) {
      const int r = lane + 64 * t;
      if (t < rt && r < rows) P[wave * ldv + r] = (TT)y[t];
    }
  }
}

// RT: row slots per lane of the panel columns (tiles of at most 64 RT rows).
template <typename TS, typename TT, int RT>
__global__ __launch_bounds__(NT) void k_qr_factor(const QrTask* __restrict__ tasks,
                                                  const QrTask* __restrict__ children, int ldv) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int rowl[MAXR];
  __shared__ int bstart[MAXR + 1];
  __shared__ double S[NB * NB];
  __shared__ double Tm[NB * NB];
  __shared__ double taus[NB];
  __shared__ double prm[8];
  const QrTask tk = tasks[blockIdx.x];
  const int m = tk.m, N = tk.ncol, tid = threadIdx.x;
  const int nf = (tk.nfact > 0 && tk.nfact < N) ? tk.nfact : N;   // factored columns
  const gptr<TT> A = glb((TT*)tk.tile);

  // ---- fill the tile (UF loads in flight per thread: clamped addresses, masked stores;
  // a tile holds fewer than 2^31 elements)
  constexpr int UF = 4;
  if (tk.nchild == 0) {
    const gptr<const TS> src = glb((const TS*)tk.src);
    const int total = m * N;
    // walk the source along its unit stride (rows of a transposed source); the (outer, inner)
    // position of element tid + j NT advances by (NT / inner, NT % inner) with a carry
    const bool by_col = tk.src_rs == 1 && tk.src_cs != 1;
    const int inner = by_col ? m : N;
    const int d_o = NT / inner, d_i = NT - d_o * inner;
    int o = tid / inner, i = tid - o * inner;
    for (int base = tid; base < total; base += UF * NT) {
      TS v[UF];
      int oo[UF], ii[UF];
#pragma unroll
      for (int k = 0; k < UF; ++k) {
        oo[k] = o;
        ii[k] = i;
        const bool in = base + k * NT < total;
        const int r = by_col ? i : o, c = by_col ? o : i;
        v[k] = src[in ? r * tk.src_rs + c * tk.src_cs : 0];
        o += d_o;
        i += d_i;
        if (i >= inner) {
          i -= inner;
          ++o;
        }
      }
#pragma unroll
      for (int k = 0; k < UF; ++k)
        if (base + k * NT < total) A[by_col ? ii[k] * N + oo[k] : oo[k] * N + ii[k]] = (TT)v[k];
    }
  } else {
    int row0 = 0;
    for (int ci = 0; ci < tk.nchild; ++ci) {
      const QrTask ch = children[tk.child0 + ci];
      const gptr<const TS> ct = glb((const TS*)ch.tile);
      const int kc = ch.m < nf ? ch.m : nf;
      const int total = kc * N;
      const int d_r = NT / N, d_c = NT - d_r * N;   // (row, column) step of NT elements
      int r = tid / N, c = tid - r * N;
      for (int base = tid; base < total; base += UF * NT) {
        TS v[UF];
        int rr[UF], cc[UF];
#pragma unroll
        for (int k = 0; k < UF; ++k) {
          v[k] = ct[(base + k * NT < total) ? base + k * NT : total - 1];
          rr[k] = r;
          cc[k] = c;
          r += d_r;
          c += d_c;
          if (c >= N) {
            c -= N;
            ++r;
          }
        }
#pragma unroll
        for (int k = 0; k < UF; ++k)
          if (base + k * NT < total)
            A[(int64_t)(row0 + rr[k]) * N + cc[k]] = (cc[k] >= rr[k] || cc[k] >= nf) ? (TT)v[k] : (TT)0;
      }
      row0 += kc;
    }
  }
  __syncthreads();

  const int kmax = m < nf ? m : nf;
  TT* P = (TT*)smem;                                       // NB columns x ldv rows
  double* scr = (double*)(smem + panel_bytes((int)sizeof(TT), ldv));
  for (int p0 = 0, pi = 0; p0 < kmax; p0 += NB, ++pi) {
    const int nb = (kmax - p0) < NB ? (kmax - p0) : NB;
    const int rows = panel_rows(rowl, bstart, m, tk.nchild, tk.kc0, tk.kc_last, p0, nb);
    for (int base = tid; base < rows * NB; base += UF * NT) {
      int ri[UF];
      TT v[UF];
#pragma unroll
      for (int k = 0; k < UF; ++k) ri[k] = rowl[((base + k * NT < rows * NB) ? base + k * NT : rows * NB - 1) >> 4];
#pragma unroll
      for (int k = 0; k < UF; ++k) {
        const int jj = (base + k * NT) & (NB - 1);
        v[k] = A[(int64_t)ri[k] * N + p0 + (jj < nb ? jj : nb - 1)];
      }
#pragma unroll
      for (int k = 0; k < UF; ++k) {
        const int idx = base + k * NT;
        if (idx < rows * NB) {
          const int r = idx >> 4, jj = idx & (NB - 1);
          P[jj * ldv + r] = (jj < nb) ? v[k] : (TT)0;
        }
      }
    }
    if (tid < NB) taus[tid] = 0.0;
    __syncthreads();
    // ---- panel columns: the smallest row-slot count that holds this panel's rows
    {
      const int rt = (rows + 63) >> 6;
      if (RT > 4 && rt <= 2) panel_columns<TT, 2>(P, ldv, rows, nb, scr, prm, taus);
      else if (RT > 4 && rt <= 4) panel_columns<TT, 4>(P, ldv, rows, nb, scr, prm, taus);
      else if (RT > 7 && rt <= 7) panel_columns<TT, 7>(P, ldv, rows, nb, scr, prm, taus);
      else if (RT > 10 && rt <= 10) panel_columns<TT, 10>(P, ldv, rows, nb, scr, prm, taus);
      else panel_columns<TT, RT>(P, ldv, rows, nb, scr, prm, taus);
    }
    __syncthreads();
    for (int idx = tid; idx < rows * NB; idx += NT) {
      const int r = idx >> 4, jj = idx & (NB - 1);
      if (jj < nb) A[(int64_t)rowl[r] * N + p0 + jj] = P[jj * ldv + r];
    }
    if (tid < nb) glb(tk.tau)[p0 + tid] = taus[tid];
    __syncthreads();
    // ---- explicit V (unit diagonal, zeros above; padded columns zero)
    if (tid < NB * NB) {
      const int jj = tid >> 4, r = tid & (NB - 1);
      if (r <= jj && r < rows) P[jj * ldv + r] = (r == jj && jj < nb) ? (TT)1 : (TT)0;
    }
    __syncthreads();
    // ---- S = V^T V on MFMA: every wave a slice of the rows, partials summed in LDS
    gram_v<TT>(P, ldv, rows, nb, scr, S);
    form_t(S, taus, Tm);
    __syncthreads();
    if (tid < NB * NB) glb((double*)tk.tmat)[(size_t)pi * NB * NB + tid] = Tm[tid];
    // ---- trailing update  A <- Q_p^T A  on the panel's rows
    // (columns beyond nf, when carried, are updated afterwards by the UPD apply kernel)
    const int c0 = p0 + nb;
    if (c0 < nf) block_update<true, TT, TT>(A, N, rowl, c0, nf, rows, P, ldv, Tm, scr);
    __syncthreads();
  }
}

// out = Q [X; Z] for one factored tile (Z the rest rows, zero when absent);
// Q = Q_0 Q_1 ... (panels applied last to first).
// Workgroup (task, y) owns the 16 output columns [16y, 16y + 16): its slice of
// W = [X; 0] stays in registers through every panel (row block b of 16 rows
// belongs to wave b mod 16; lane l holds rows 4s + l/16 of the block, column
// l%16, in the B-operand layout of K-step s), so the only memory traffic per
// panel is the panel's V, staged in LDS by tile row with zeros on the rows the
// panel does not touch.  Per panel: W_p = V^T W (per-wave MFMA partials summed
// in LDS in wave order), Y = T W_p, W -= V Y.
// UPD: the trailing update of a column block instead, in place: the columns
// out[r * out_rs + c * out_cs] (c < t, r < m, tile dtype) are replaced by
// Q^T times them (panels first to last, Y = T^T W_p), one workgroup per 16 of them.
template <typename TT, typename TO, bool UPD>
__global__ __launch_bounds__(NT) void k_qr_apply(const ApplyTask* __restrict__ tasks, int ldv) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int bstart[MAXR + 1];
  __shared__ double Tm[NB * NB];
  __shared__ double wsum[NB * NB];
  typedef Mma<TT> M;
  const ApplyTask tk = tasks[blockIdx.x];
  const int m = tk.m, N = tk.ncol, t = tk.t, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cb = blockIdx.y * NB;
  if (cb >= t) return;   // the whole workgroup: no barrier is reached
  const int col = cb + (lane & 15);
  const bool colok = col < t;
  const gptr<const TT> tile = glb((const TT*)tk.tile);
  const gptr<const double> X = glb(tk.x);
  TT* V = (TT*)smem;   // [NB][ldv], ldv > m: row index = tile row
  double* wpart = (double*)(smem + panel_bytes((int)sizeof(TT), ldv));
  constexpr int RB = (MAXR / NB + NWV - 1) / NWV;
  const int nrb = (m + NB - 1) / NB;
  double Wr[RB][4];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int row = (wave + NWV * b) * NB + 4 * s + (lane >> 4);
      double v = 0.0;
      if (UPD) {
        if (colok && row < m) v = (double)glb((const TT*)tk.out)[(int64_t)row * tk.out_rs + (int64_t)col * tk.out_cs];
      } else if (colok && row < tk.k_in) {
        v = X[(int64_t)row * tk.x_ld + col];
      } else if (colok && row < m && tk.rest) {
        v = tk.rest[(int64_t)(row - tk.k_in) * tk.rest_ld + col];
      }
      Wr[b][s] = v;
    }
  const int np = (tk.kq + NB - 1) / NB;
  for (int it = 0; it < np; ++it) {
    const int pi = UPD ? it : np - 1 - it;
    const int p0 = pi * NB;
    const int nb = (tk.kq - p0) < NB ? (tk.kq - p0) : NB;
    // node: first compacted row index of each child block's active rows
    if (tk.nchild > 0 && tid == 0) {
      int c = 0;
      for (int b = 0; b < tk.nchild; ++b) {
        const int off = b * tk.kc0;
        const int kcb = (b == tk.nchild - 1) ? tk.kc_last : tk.kc0;
        const int lo = (p0 - off) > 0 ? (p0 - off) : 0;
        const int hi = kcb < (p0 + nb) ? kcb : (p0 + nb);
        bstart[b] = c;
        c += (hi > lo) ? (hi - lo) : 0;
      }
    }
    __syncthreads();   // also: every wave is done with the previous panel's V, T and partials
    if (tid < NB * NB) Tm[tid] = glb((const double*)tk.tmat)[(size_t)pi * NB * NB + tid];
    // V by tile row: compacted index r of an active row (reflector jj has its unit
    // entry at r == jj and its stored entries at r > jj), zero elsewhere
    constexpr int UF = 4;   // loads in flight per thread (clamped addresses, masked values)
    for (int base = tid; base < m * NB; base += UF * NT) {
      int rr[UF];
      TT v[UF];
#pragma unroll
      for (int k = 0; k < UF; ++k) {
        const int idx = (base + k * NT < m * NB) ? base + k * NT : m * NB - 1;
        const int row = idx >> 4;
        int r = -1;
        if (tk.nchild == 0) {
          r = row - p0;
        } else {
          int b = row / tk.kc0;
          if (b > tk.nchild - 1) b = tk.nchild - 1;
          const int off = b * tk.kc0;
          const int kcb = (b == tk.nchild - 1) ? tk.kc_last : tk.kc0;
          const int i = row - off;
          const int lo = (p0 - off) > 0 ? (p0 - off) : 0;
          const int hi = kcb < (p0 + nb) ? kcb : (p0 + nb);
          if (i >= lo && i < hi) r = bstart[b] + (i - lo);
        }
        rr[k] = r;
        const int jj = idx & (NB - 1);
        v[k] = tile[(int64_t)row * N + p0 + (jj < nb ? jj : nb - 1)];
      }
#pragma unroll
      for (int k = 0; k < UF; ++k) {
        const int idx = base + k * NT;
        if (idx < m * NB) {
          const int row = idx >> 4, jj = idx & (NB - 1);
          const int r = rr[k];
          V[jj * ldv + row] = (jj < nb && r >= jj) ? ((r == jj) ? (TT)1 : v[k]) : (TT)0;
        }
      }
    }
    __syncthreads();
    // W_p partial over this wave's row blocks
    typename M::acc_t w = M::zero();
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int rb = wave + NWV * b;
      if (rb < nrb) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int row = rb * NB + 4 * s + (lane >> 4);
          const TT a = row < m ? V[(lane & 15) * ldv + row] : (TT)0;
          w = M::mma(a, (TT)Wr[b][s], w);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) wpart[wave * 256 + v * 64 + lane] = (double)w[v];
    __syncthreads();
    // W_p: thread e < 256 sums element e of the partials in wave order
    if (tid < 256) {
      double a = 0.0;
      for (int p = 0; p < NWV; ++p) a += wpart[p * 256 + tid];
      wsum[tid] = a;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) w[v] = (TT)wsum[v * 64 + lane];
    // Y = T W_p (Q applied), Y = T^T W_p (Q^T applied)
    typename M::acc_t y = M::zero();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = lane & 15, k = 4 * s + (lane >> 4);
      y = M::mma((TT)(UPD ? Tm[k * NB + i] : Tm[i * NB + k]), bop(w, s), y);
    }
    TT yb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) yb[s] = bop(y, s);
    // W -= V Y on this wave's row blocks
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int rb = wave + NWV * b;
      if (rb < nrb) {
        const int ra = rb * NB + (lane & 15);
        typename M::acc_t d = M::zero();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const TT a = ra < m ? V[(4 * s + (lane >> 4)) * ldv + ra] : (TT)0;
          d = M::mma(a, yb[s], d);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) Wr[b][s] -= (double)bop(d, s);
      }
    }
  }
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int row = (wave + NWV * b) * NB + 4 * s + (lane >> 4);
      if (colok && row < m) {
        if (UPD) glb((TT*)tk.out)[(int64_t)row * tk.out_rs + (int64_t)col * tk.out_cs] = (TT)Wr[b][s];
        else if (tk.to_out == 2) glb((double*)tk.out)[row * tk.out_rs + col * tk.out_cs] = Wr[b][s];
        else if (tk.to_out) glb((TO*)tk.out)[row * tk.out_rs + col * tk.out_cs] = (TO)Wr[b][s];
        else glb(tk.work)[(int64_t)row * t + col] = Wr[b][s];
      }
    }
}

size_t panel_smem(int elt, int ldv) { return panel_bytes(elt, ldv) + (size_t)SCR_DOUBLES * 8; }

template <typename K>
hipError_t raise_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

// smallest instantiated row-slot count that holds max_rows (unconditional
// loads of the published column then read no slot past the tile)
constexpr int RT_MAX = (MAXR + 63) / 64;
static_assert(RT_MAX == 13, "row-slot buckets below assume 800-row tiles");
template <typename TS, typename TT>
void launch_factor_rt(int max_rows, dim3 grid, dim3 block, size_t sm, hipStream_t s, const QrTask* t,
                      const QrTask* c, int ldv) {
  const int rt = (max_rows + 63) / 64;
  if (rt <= 4) hipLaunchKernelGGL((k_qr_factor<TS, TT, 4>), grid, block, sm, s, t, c, ldv);
  else if (rt <= 7) hipLaunchKernelGGL((k_qr_factor<TS, TT, 7>), grid, block, sm, s, t, c, ldv);
  else if (rt <= 10) hipLaunchKernelGGL((k_qr_factor<TS, TT, 10>), grid, block, sm, s, t, c, ldv);
  else hipLaunchKernelGGL((k_qr_factor<TS, TT, RT_MAX>), grid, block, sm, s, t, c, ldv);
}

hipError_t launch_qr_factor(int dtype_src, int dtype_tile, const QrTask* d_tasks, const QrTask* d_children,
                            int ntasks, int max_rows, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  if (max_rows > MAXR) return hipErrorInvalidValue;
  const int ldv = max_rows + 1;
  dim3 grid(ntasks), block(NT);
  if (dtype_tile == 0) {
    const size_t sm = panel_smem(8, ldv);
    if (dtype_src == 0) launch_factor_rt<double, double>(max_rows, grid, block, sm, s, d_tasks, d_children, ldv);
    else launch_factor_rt<float, double>(max_rows, grid, block, sm, s, d_tasks, d_children, ldv);
  } else {
    const size_t sm = panel_smem(4, ldv);
    launch_factor_rt<float, float>(max_rows, grid, block, sm, s, d_tasks, d_children, ldv);
  }
  return hipGetLastError();
}

hipError_t launch_qr_apply(int dtype_tile, int dtype_out, const ApplyTask* d_tasks, int ntasks, int max_rows,
                           int max_t, hipStream_t s) {
  if (ntasks <= 0 || max_t <= 0) return hipSuccess;
  if (max_rows > MAXR) return hipErrorInvalidValue;
  const int ldv = max_rows + 1;
  dim3 grid(ntasks, (max_t + NB - 1) / NB), block(NT);
  if (dtype_tile == 0) {
    const size_t sm = panel_smem(8, ldv);
    if (dtype_out == 0) hipLaunchKernelGGL((k_qr_apply<double, double, false>), grid, block, sm, s, d_tasks, ldv);
    else hipLaunchKernelGGL((k_qr_apply<double, float, false>), grid, block, sm, s, d_tasks, ldv);
  } else {
    const size_t sm = panel_smem(4, ldv);
    if (dtype_out == 0) hipLaunchKernelGGL((k_qr_apply<float, double, false>), grid, block, sm, s, d_tasks, ldv);
    else hipLaunchKernelGGL((k_qr_apply<float, float, false>), grid, block, sm, s, d_tasks, ldv);
  }
  return hipGetLastError();
}

hipError_t launch_qr_update(int dtype_tile, const ApplyTask* d_tasks, int ntasks, int max_rows, int max_t,
                            hipStream_t s) {
  if (ntasks <= 0 || max_t <= 0) return hipSuccess;
  if (max_rows > MAXR) return hipErrorInvalidValue;
  const int ldv = max_rows + 1;
  dim3 grid(ntasks, (max_t + NB - 1) / NB), block(NT);
  if (dtype_tile == 0)
    hipLaunchKernelGGL((k_qr_apply<double, double, true>), grid, block, panel_smem(8, ldv), s, d_tasks, ldv);
  else
    hipLaunchKernelGGL((k_qr_apply<float, float, true>), grid, block, panel_smem(4, ldv), s, d_tasks, ldv);
  return hipGetLastError();
}

template <typename TS, typename TT>
hipError_t raise_factor(size_t bytes) {
  hipError_t e;
  if ((e = raise_lds(k_qr_factor<TS, TT, 4>, bytes)) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_factor<TS, TT, 7>, bytes)) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_factor<TS, TT, 10>, bytes)) != hipSuccess) return e;
  return raise_lds(k_qr_factor<TS, TT, RT_MAX>, bytes);
}

hipError_t qr_kernels_init() {
  hipError_t e;
  const size_t s8 = panel_smem(8, MAXR + 1), s4 = panel_smem(4, MAXR + 1);
  if ((e = raise_factor<double, double>(s8)) != hipSuccess) return e;
  if ((e = raise_factor<float, double>(s8)) != hipSuccess) return e;
  if ((e = raise_factor<float, float>(s4)) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_apply<double, double, false>, s8)) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_apply<double, float, false>, s8)) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_apply<float, double, false>, s4)) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_apply<float, float, false>, s4)) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_apply<double, double, true>, s8)) != hipSuccess) return e;
  if ((e = raise_lds(k_qr_apply<float, float, true>, s4)) != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace tto
