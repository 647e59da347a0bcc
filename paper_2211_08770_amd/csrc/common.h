// Internal declarations shared by the HIP kernels and the host library.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace tto {

// ---------------------------------------------------------------------------
// Householder QR of one tile (TSQR leaf or tree node).
//
// The tile is row-major m x ncol (ld = ncol).  After factorisation its upper
// triangle holds R and the strict lower part holds the Householder vectors
// (unit leading entry implied); tau[j] and, per panel of QR_NB reflectors,
// the upper-triangular T of the compact WY form I - V T V^T are stored beside it.
// ---------------------------------------------------------------------------
constexpr int QR_NB = 16;          // panel width
constexpr int QR_THREADS = 1024;   // 16 waves per tile
constexpr int QR_MAXROWS = 800;    // LDS panel: QR_MAXROWS x QR_NB doubles = 100 KiB (fan-in 4 at 200 columns)
constexpr int QR_BLOCK_COLS = 384; // columns per block of a column-blocked QR (fan-in 2, 768-row tiles)

struct QrTask {
  const void* src;        // leaf: element (r, c) at src[r * src_rs + c * src_cs]
  int64_t src_rs, src_cs;
  int32_t nchild;         // > 0: tree node stacking the R factors of children[child0 ..]
  int32_t child0;
  int32_t kc0, kc_last;   // node: rows contributed by each child but the last, and by the last
  int32_t m, ncol;        // tile shape
  void* tile;             // row-major m x ncol
  double* tau;            // [min(m, nfact)]
  void* tmat;             // [npanels][QR_NB][QR_NB] doubles: T of each panel (I - V T V^T)
  int32_t nfact;          // columns factored (0: all); the columns beyond are carried and
                          // updated by the reflectors (a column block of a blocked QR).  A node
                          // then stacks the top min(m, nfact) rows of each child: triangular in
                          // the factored columns, full in the carried ones.
};

// Apply the orthogonal factor of a factored tile:  out = Q * [X; Z].
// X is k_in x t (double, row-major, ld = x_ld); Z holds the rows k_in..m-1 (double,
// row-major, ld = rest_ld) or is zero when rest is null; out is m x t.
struct ApplyTask {
  const void* tile;       // factored tile (V below the diagonal), ld = ncol
  const double* tau;
  const void* tmat;
  int32_t m, ncol, kq;    // kq = number of reflectors = min(m, ncol)
  int32_t nchild, kc0, kc_last;   // node structure (stacked triangles); nchild = 0 for a dense leaf
  int32_t k_in, t;
  const double* x;
  int64_t x_ld;
  double* work;           // m x t row-major scratch (tree nodes keep their result here)
  void* out;              // leaves: final destination (out dtype), strides below
  int64_t out_rs, out_cs;
  int32_t to_out;         // 1: write to out (with cast); 2: write to out as double; 0: result stays in work
  const double* rest;     // rows k_in..m-1 of the input (null: zero)
  int64_t rest_ld;
};

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD of a (kr x ncol) upper-trapezoidal R factor, FP64.
// ---------------------------------------------------------------------------
constexpr int SVD_SMALL_MAX = 1024;  // R factors of at most this many rows: one workgroup per SVD
constexpr int SVD_BIG_MAX = 4096;    // above: block Jacobi over many workgroups, up to this many rows
constexpr int SVD_BLOCK_MIN = 224;   // default crossover: block Jacobi above this many rows (measured: the
                                     // one-workgroup kernel is faster at 128 rows, half as fast at 256)
struct SvdTask {
  const void* R;          // row-major kr x ncol, ld = r_ld (root tile of a TSQR)
  int64_t r_ld;
  int32_t r_f32;          // 1: R is float (root of a one-tile FP32 tree), 0: double
  int32_t kr, ncol;
  int32_t upper;          // 1: R is upper trapezoidal (entries below the diagonal read as 0)
  double bulk_u;          // unit round-off of the arithmetic that produced R (deflation scale; 0: none)
  double* A;              // scratch ncol x kr, column-major
  double* acc;            // scratch kr x kr, column-major
  double* sigma;          // [kr] sorted decreasing on exit
  int32_t* perm;          // [kr] scratch
  const double* norm;     // device ||x||; eps = delta / sqrt(d-1) * norm
  double delta_scaled;    // delta / sqrt(d-1)
  double eps_floor;       // eps = max(delta_scaled, eps_floor) * norm (FP32-bulk noise floor; 0 in FP64)
  int64_t max_rank;       // <= 0: none
  int32_t* rank_out;      // device int
  double* wt;             // ncol x t row-major:  W^T  with W = Sigma_t V_t^T
  double* ur;             // kr x t row-major:  left factor fed to Q application
  int32_t t_ld;           // > 0: wt and ur have t_ld columns (a bound of the rank), zero beyond t
  int32_t* info;          // device int: sweeps used (diagnostic)
  int32_t block;          // 1: block Jacobi over many workgroups (launch_svd_big), 0: one workgroup (launch_svd)
  int32_t* iscr;          // block: int scratch of 2 kr + 128 entries
};

// ---------------------------------------------------------------------------
// Batched GEMM used by the right-to-left contraction:
//   C[r][c] = sum_parts coef_p * sum_k A_p[r][k] * B[c][b_off_p + k]
// A_p row-major (M x K_p, ld = K_p, dtype T); B row-major double (ld = b_ld);
// C row-major (M x N, ld = c_ld, dtype T).
// ---------------------------------------------------------------------------
struct GemmPart {
  const void* A;
  int32_t K;
  int32_t b_off;
  double coef;
};

struct GemmTask {
  int32_t M, N;
  int32_t part0, nparts;
  const void* B;          // entries B[c][j] with j < c read as zero (R factor of a tile)
  int64_t b_ld;
  int32_t b_f32;          // 1: B is float (root of a one-tile FP32 tree), 0: double
  void* C;
  int64_t c_ld;
};

// Strided GEMM C = A B (A, C in the tile dtype, B double) for the left-to-right
// contraction with an explicitly formed orthogonal factor:
//   C[r*c_rs + c*c_cs] = sum_k A[r*a_rs + k*a_cs] * B[k*b_rs + c*b_cs]
struct GemmSTask {
  const void* A;
  int64_t a_rs, a_cs;
  const double* B;
  int64_t b_rs, b_cs;
  void* C;
  int64_t c_rs, c_cs;
  int32_t M, N, K;
};
hipError_t launch_gemm_strided(int dtype, const GemmSTask* d_tasks, int ntasks, int max_m, int max_n, hipStream_t s);
// X = identity (n x n, row-major, ld = n)
hipError_t launch_eye(double* X, int n, hipStream_t s);

// ---------------------------------------------------------------------------
// TT inner product of one pair of components (left-to-right contraction).
// ---------------------------------------------------------------------------
struct DotTask {
  int32_t d;
  const void* x;          // packed cores
  const void* y;
  const int64_t* nn;      // device [d] mode sizes
  const int64_t* rx;      // device [d+1] ranks of x
  const int64_t* ry;      // device [d+1] ranks of y
  double coef;
  void* w;                // scratch 2 * wcap doubles (FP64 for both input dtypes)
  int64_t wcap;           // >= max_k rx_k * ry_k
  void* tmp;              // scratch >= max_k rx_k * n_k * ry_{k+1} doubles
  double* out;            // result slot: coef * <x, y>
};

// Batched copy of row-major blocks between dtypes (column-blocked QR: trailing
// rows of the tiles gathered into the next block's matrix, R factors assembled):
//   dst[r * dst_ld + c] = (src && !(tri && c < r)) ? src[r * src_ld + c] : 0
struct BlockCopy {
  const void* src;
  int64_t src_ld;
  void* dst;
  int64_t dst_ld;
  int32_t rows, cols;
  int32_t src_f32, dst_f32;
  int32_t tri;            // 1: entries left of the diagonal written as zero
};
hipError_t launch_block_copy(const BlockCopy* d_tasks, int ntasks, int64_t max_rows, hipStream_t s);

// Batched strided copy: dst[i] = coef * src[i] (+ dst[i] when accumulate).
struct CopySeg {
  const void* src;
  void* dst;
  int64_t count;
  double coef;
  int32_t accumulate;
};

// ---------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files).
// ---------------------------------------------------------------------------
hipError_t launch_qr_factor(int dtype_src, int dtype_tile, const QrTask* d_tasks, const QrTask* d_children,
                            int ntasks, int max_rows, hipStream_t s);
hipError_t launch_qr_apply(int dtype_tile, int dtype_out, const ApplyTask* d_tasks, int ntasks, int max_rows,
                           int max_t, hipStream_t s);
// Trailing update of column blocks: tile columns out[r * out_rs + c * out_cs] (c < t,
// r < m, tile dtype) replaced in place by Q^T times them (Q the tile's reflectors).
hipError_t launch_qr_update(int dtype_tile, const ApplyTask* d_tasks, int ntasks, int max_rows, int max_t,
                            hipStream_t s);
hipError_t launch_svd(const SvdTask* d_tasks, int ntasks, hipStream_t s);
// The tasks with the block flag (the others are skipped): block Jacobi, several launches;
// max_kr bounds kr over the flagged tasks.  Every sweep's rounds are launched (sized by
// max_kr; the rounds of a converged task return at once), so nothing waits for the host.
hipError_t launch_svd_big(const SvdTask* d_tasks, int ntasks, int max_kr, hipStream_t s);
hipError_t launch_gemm(int dtype, const GemmTask* d_tasks, const GemmPart* d_parts, int ntasks,
                       int max_m, int max_n, hipStream_t s);
hipError_t launch_dot(int dtype, const DotTask* d_tasks, int ntasks, hipStream_t s);
hipError_t launch_sumsq(int dtype, const void* x, int64_t n, double* out_norm, hipStream_t s);
// Frobenius norms of several buffers in one launch (one workgroup per buffer).
struct SumsqTask {
  const void* x;
  int64_t n;
  double* out;
};
hipError_t launch_sumsq_batched(int dtype, const SumsqTask* d_tasks, int ntasks, hipStream_t s);
hipError_t launch_scale(int dtype, void* x, int64_t n, const double* d_norm, hipStream_t s);
hipError_t launch_copy_segs(int dtype, const CopySeg* d_segs, int nsegs, hipStream_t s);
// out[idx ? idx[o] : o] = sum of slots[seg[o] .. seg[o+1])
hipError_t launch_segsum(const double* slots, const int32_t* seg, const int32_t* idx, int nout, double* out,
                         hipStream_t s);
hipError_t launch_cholinv(double* G, int m, double* Rinv, int32_t* info, double u, hipStream_t s);
// Leading blocks of G packed: E_k = I - G_k (minus_identity = 1) or G_k (0).
hipError_t launch_loo_mats(const double* G, int m, double* E, int minus_identity, hipStream_t s);

// z core = alpha*x core (+) y core in the TT-sum layout (block concatenation).
struct AxpyTask {
  const void* x;
  const void* y;
  void* z;
  int32_t n;
  int32_t xr0, xr1, yr0, yr1;  // ranks of the x / y cores
  int32_t first, last;         // first core: rows shared; last core: columns shared
  double alpha;                // applied to x (first core only)
};
hipError_t launch_axpy(int dtype, const AxpyTask* d_tasks, int ntasks, int64_t max_elems, hipStream_t s);

// Small FP64 updates of the scheme drivers (single thread, sequential order):
//   MGS correction   r[j] = dots[j] - sum_{l<j} r[l] * Gq[l*ldg + j]   (j < i)
//   negated copy     coef[j] = -r[j]
// Projection coefficients of one pass of a Gram-Schmidt step, for a batch of
// requests (one thread per request, sequential in j):
//   CGS: r[j] = dots[j];   MGS: r[j] = dots[j] - sum_{l<j} r[l] * gram[l*b + j]
// (gram null: the identity).
struct CoefTask {
  const double* dots;
  const double* gram;
  double* r;
  int32_t b;
  int32_t modified;
};
hipError_t launch_fill_pattern(int dtype, void* x, int64_t n, hipStream_t s);
// Cores of a rounding planned at rank bounds tb_k, held at their bound shapes in a staging
// buffer, copied into the packed result at the ranks the device chose (one workgroup per job).
// geo: [d] n_k, [d+1] tb_k, [d] staging offsets.  ranks[1..d-1] are read; ranks[0] and
// ranks[d] are set to 1.  status is set to TT_ECAPACITY (-3) when the result exceeds capacity.
struct CompactTask {
  const void* staging;
  void* out;
  int64_t capacity;
  const int64_t* geo;
  int32_t* ranks;
  int32_t* status;
  int32_t d;
  int32_t active;         // 0: only ranks[0] = ranks[d] = 1 (order one or a failed job)
  int32_t init_status;    // the job's status as the host decided it, written to *status first
};
hipError_t launch_compact(int dtype, const CompactTask* d_tasks, int ntasks, hipStream_t s);
hipError_t launch_coef_batched(const CoefTask* d_tasks, int ntasks, hipStream_t s);

hipError_t launch_mgs_correct(const double* dots, const double* Gq, int ldg, int i, double* r, double* neg,
                              hipStream_t s);
// TT-Householder (Algorithms 6-8): canonical rank-one TT-vectors e_first..e_{first+count-1}
// (S = sum_k n_k elements each, d_n on the device), column i of R with the
// coefficients of the Householder sum, the reflection coefficients of the later
// vectors by u_i and the coefficients of every q_i, both in component form over
// the Gram matrix of the Householder vectors.
hipError_t launch_canonical(int dtype, void* out, const int64_t* d_n, int d, int64_t S, int64_t first, int count,
                            hipStream_t s);
hipError_t launch_hh_column(const double* dots, int i, int norm_given, double* Rcol, double* coef, hipStream_t s);
hipError_t launch_hh_reflect(const double* dots_a, const double* G, double* Ct, int m, int i, hipStream_t s);
hipError_t launch_hh_qcoef(const double* EU, const double* G, double* D, int m, hipStream_t s);
// One core of y = alpha * Delta_d x (Dirichlet Laplacian as a rank-two TT-matrix);
// kind 0 first, 1 interior, 2 last, 3 only core.  x[0..n) = v.
hipError_t launch_laplacian_core(int dtype, const void* X, int64_t r0, int64_t n, int64_t r1, int kind, double alpha,
                                 void* Y, hipStream_t s);
hipError_t launch_fill_const(int dtype, void* x, int64_t n, double v, hipStream_t s);
// y[0..n) = x[0..n) converted from src_dtype to dst_dtype (0 f64, 1 f32)
hipError_t launch_cast(int src_dtype, const void* x, int dst_dtype, void* y, int64_t n, hipStream_t s);
// out[j] = a[j] + b[j]
hipError_t launch_add(const double* a, const double* b, double* out, int n, hipStream_t s);
hipError_t launch_neg(const double* a, double* out, int n, hipStream_t s);
// Symmetrise a Gram matrix filled on (i, j), j <= i: G[j][i] = G[i][j].
hipError_t launch_sym_lower(double* G, int m, hipStream_t s);
// out[i*m + j] = L[i*m + j] for j <= i, else 0
hipError_t launch_tril(const double* L, int m, double* out, hipStream_t s);

hipError_t qr_kernels_init();   // raise LDS limits, once per process

}  // namespace tto
