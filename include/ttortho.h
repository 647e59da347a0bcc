/*
 * ttortho.h - C ABI of the MI355X (gfx950) TT-rounding / TT-orthogonalization library.
 *
 * Implements, for tensors in Tensor-Train (TT) format, the operations of
 * Coulaud, Giraud & Iannacito, "On some orthogonalization schemes in Tensor
 * Train format" (Inria RR-9491):
 *   - TT inner product and TT sum/axpy            (Section 2, TT-format)
 *   - TT-round(x, delta)                          (Section 2; rounding algorithm cited there)
 *   - TT-CGS, TT-MGS, TT-CGS2, TT-MGS2, TT-Gram   (Section 3, Algorithms 1-5)
 *   - loss of orthogonality ||I - Q^T Q||_2       (Section 3.4, equation LOO)
 *
 * Conventions shared by every entry point
 *   - Tensor data are DEVICE pointers on the context's device; every call is
 *     ordered on the context's HIP stream and returns after that stream has
 *     completed the call's work (so host-side outputs are valid on return),
 *     except tt_round_batched_async and tt_dot_noalloc, which return once
 *     their work is enqueued (their declarations say when results are valid).
 *   - A TT-vector of order d stores core k (k = 0..d-1) row-major as
 *     [r_k][n_k][r_{k+1}] at element offset sum_{j<k} r_j n_j r_{j+1};
 *     r_0 = r_d = 1.  Its left unfolding ((r_k n_k) x r_{k+1}) and its right
 *     unfolding (r_k x (n_k r_{k+1})) are both plain row-major views.
 *   - dtype TT_F64: all arithmetic in double.  dtype TT_F32 ("FP32-bulk"):
 *     cores are float and the bulk QR panels and contractions run in float,
 *     while R factors of the QR trees, the small SVDs, norms, thresholds,
 *     Gram/Cholesky steps and orthogonality measures are double.
 *   - The caller owns every buffer.  Outputs never alias inputs.  The library
 *     works inside the workspace attached to the context (see
 *     tt_ctx_set_workspace) and never allocates or frees caller memory; it
 *     keeps only a few small internal device/pinned buffers per context.
 *   - Errors are returned as tt_status; nothing is thrown across the ABI.
 *     Argument errors are detected before any device work.  On error the
 *     contents of outputs are undefined.  tt_last_error() gives a message.
 */
#ifndef TTORTHO_H
#define TTORTHO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_MAXD 64

typedef enum {
  TT_OK = 0,
  TT_EINVAL = -1,       /* bad argument (shape, rank, dtype, delta, pointer)            */
  TT_ENOMEM = -2,       /* internal small buffer could not be allocated                */
  TT_ECAPACITY = -3,    /* workspace or output capacity too small (see tt_last_error)   */
  TT_ENOTSPD = -4,      /* Gram matrix not positive definite (Section 3.2, remark)      */
  TT_EBREAKDOWN = -5,   /* ||p|| = 0 in a Gram-Schmidt scheme (dependent inputs)        */
  TT_ENONFINITE = -6,   /* NaN or Inf met in the data                                   */
  TT_EDEVICE = -7,      /* HIP runtime error                                            */
  TT_EGUARD = -8,       /* pre-round rank exceeded the caller's guard                   */
  TT_ENOTIMPL = -9
} tt_status;

typedef enum { TT_F64 = 0, TT_F32 = 1 } tt_dtype;

typedef enum { TT_CGS = 0, TT_MGS = 1, TT_CGS2 = 2, TT_MGS2 = 3, TT_GRAM = 4, TT_HOUSEHOLDER = 5 } tt_scheme;

/* One TT-vector (Section 2, TT representation).  Host struct, device data. */
typedef struct tt_vec {
  int32_t d;                  /* order, 1 <= d <= TT_MAXD                                */
  int32_t dtype;              /* tt_dtype                                                */
  int64_t n[TT_MAXD];         /* mode sizes n_0..n_{d-1} >= 1                            */
  int64_t r[TT_MAXD + 1];     /* ranks r_0..r_d with r_0 = r_d = 1; written for outputs  */
  void* data;                 /* device pointer to the packed cores                      */
  int64_t capacity;           /* elements available at data (checked for outputs)        */
} tt_vec;

/* Lazy TT sum  sum_c coef[c] * comp[c]  (Section 2: TT addition, ranks add).
 * Never materialised: rounding reads the components directly and uses the
 * block structure of the sum.  coef is a HOST array. */
typedef struct tt_sum {
  int32_t ncomp;
  const double* coef;
  const tt_vec* comp;
} tt_sum;

/* Per-call statistics of tt_orthogonalize. */
typedef struct tt_ortho_stats {
  int32_t rounds;             /* TT-round calls made (Table 1: m, m, 2m, 2m, m)           */
  int32_t m_reached;          /* vectors completed before any error                      */
  int32_t max_pre_rank;       /* largest bond rank of a vector before rounding           */
  int32_t max_post_rank;      /* largest bond rank of a vector after rounding            */
  int64_t* q_pre_size;        /* caller HOST array [m] or NULL: packed size (elements) of
                                 the lazy sum whose rounding gave q_i, i.e. the TT storage
                                 before that compression; with the packed size of q_i it
                                 gives the compression gain of Section 2 (a ratio of the
                                 compression ratios before and after rounding)             */
} tt_ortho_stats;

typedef struct tt_ctx tt_ctx;

/* Create a context bound to HIP device `device` and stream `stream`
 * (a hipStream_t, or NULL for the default stream).  Allocates a few KB of
 * device and pinned host memory for ranks, norms and status words. */
tt_status tt_ctx_create(tt_ctx** ctx, int device, void* stream);
void tt_ctx_destroy(tt_ctx* ctx);

/* Attach caller-owned device workspace (bytes, 256-byte aligned pointer).
 * Every compute call checks that its need fits; otherwise TT_ECAPACITY and
 * tt_ctx_required_bytes() tells the size that is needed. */
tt_status tt_ctx_set_workspace(tt_ctx* ctx, void* workspace, size_t bytes);
size_t tt_ctx_required_bytes(const tt_ctx* ctx);

/* Per-launch timing of this context (tracing support).  When on, every kernel
 * launch is bracketed by HIP events on the context's stream and, per kind of
 * kernel (0 qr_factor_leaf, 1 qr_factor_node, 2 qr_apply, 3 svd_jacobi,
 * 4 contraction_gemm, 5 tt_dot, 6 other), the elapsed milliseconds, launch
 * count and algorithmic flops and bytes of the launched work are summed.
 * tt_ctx_set_profiling resets the sums. */
tt_status tt_ctx_set_profiling(tt_ctx* ctx, int on);
tt_status tt_ctx_profile(const tt_ctx* ctx, int kind, double* ms, int64_t* launches, double* flops,
                         double* bytes);
const char* tt_profile_kind_name(int kind);

/* Autotuning of the TSQR tree shapes (rows of a leaf tile, children per tree
 * node).  When on, a TT-round call first times a few candidate shapes on
 * synthetic data for every QR shape class it has not met before (dtype,
 * columns, ceil(log2 rows)) and keeps the fastest for the rest of the
 * process; results do not depend on the shape, only the time does. */
tt_status tt_ctx_set_autotune(tt_ctx* ctx, int on);
/* Tune one shape class now; leaf_rows and fanin (nullable) receive the choice.
 * Needs workspace for a rows x cols matrix and its tree (TT_ECAPACITY otherwise). */
tt_status tt_tune_tsqr(tt_ctx* ctx, int64_t rows, int64_t cols, int32_t dtype, int32_t* leaf_rows, int32_t* fanin);

/* Human-readable status and last error message of this context. */
const char* tt_status_str(tt_status s);
const char* tt_last_error(const tt_ctx* ctx);

/* <x, y> for two lazy sums (Section 2, Euclidean inner product; used by every
 * algorithm of Section 3).  Computed as sum over component pairs of
 * coef * coef' * <x_c, y_c'>, each by the left-to-right contraction
 * W_k = sum_i X_k(i)^T W_{k-1} Y_k(i) on the FP64 matrix cores: FP32 cores are
 * widened exactly, so for either dtype every product and sum is FP64.
 * out: HOST double. */
tt_status tt_dot(tt_ctx* ctx, const tt_sum* x, const tt_sum* y, double* out);

/* npairs inner products <xs[p], ys[p]> in one batched launch. out: HOST [npairs]. */
tt_status tt_dot_batched(tt_ctx* ctx, int32_t npairs, const tt_sum* xs, const tt_sum* ys,
                         double* out);

/* z = alpha * x + y materialised (Section 2: first core concatenated
 * horizontally, middle cores block diagonal, last core vertically; ranks add).
 * alpha multiplies x's first core.  z->r is written; z->capacity must be at
 * least the packed size of the result. */
tt_status tt_axpy(tt_ctx* ctx, double alpha, const tt_vec* x, const tt_vec* y, tt_vec* z);

/* ||x|| of a lazy sum (Section 2: Frobenius norm of the full tensor),
 * computed stably by the right-to-left QR sweep of TT-round: after it,
 * ||x|| = ||G_0||_F.  With a sum x + (-1) y this gives ||x - y|| without the
 * cancellation of sqrt(<x,x> - 2<x,y> + <y,y>).  out: HOST double. */
tt_status tt_norm(tt_ctx* ctx, const tt_sum* x, double* out);

/* TT-round(x, delta) (Section 2): returns x~ with ||x - x~|| <= delta ||x||.
 * Right-to-left QR sweep, then left-to-right truncated SVD at per-bond
 * threshold delta / sqrt(d-1) * ||x||, keeping the smallest rank whose
 * discarded tail is <= the threshold (and <= max_rank when max_rank > 0).
 * Cores 0..d-2 of the result are left-orthonormal.  d = 1 copies; a zero
 * tensor yields all ranks 1 (unit-vector cores 0..d-2, zero last core).  out->r is written; norm_x (HOST, nullable)
 * receives ||x||.  Unfoldings of any width are factored (in column blocks of 384 when
 * they have more than 800 rows and 400 columns); a left-to-right R factor of more than
 * 4096 rows gives TT_ENOTIMPL. */
tt_status tt_round(tt_ctx* ctx, const tt_sum* x, double delta, int64_t max_rank, tt_vec* out,
                   double* norm_x);

/* njobs independent roundings in shared batched launches (jobs may differ in
 * d, n, ranks and component count).  deltas, max_ranks (nullable) and
 * job_status are HOST arrays of length njobs. */
tt_status tt_round_batched(tt_ctx* ctx, int32_t njobs, const tt_sum* xs, const double* deltas,
                           const int64_t* max_ranks, tt_vec* outs, tt_status* job_status);

/* tt_round_batched without waiting: every left-to-right step is planned at the
 * rank bounds min(t_{k-1} n_{k-1}, s_k, max_rank) (rows and columns beyond the
 * rank the device chooses are zero), the result cores are formed at those bound
 * shapes in the workspace and compacted into outs[j] on the device at the ranks
 * it chose, so no step waits for the host (the synchronous call reads every rank
 * back to plan the next step at it).  Same results as tt_round_batched where the
 * output ranks equal the bounds (bitwise); otherwise equal up to rounding, at the
 * cost of the padded rows.  The call returns once all work is enqueued on the
 * context's stream; ranks (HOST pinned int32 [njobs * (TT_MAXD + 1)]: the ranks
 * of job j at ranks[j * (TT_MAXD + 1) + k], k = 0..d), job_status (HOST pinned
 * int32 [njobs]: TT_OK, or TT_ECAPACITY when outs[j] cannot hold the result) and
 * norms (HOST pinned double [njobs] or NULL: ||x_j||) are filled by copies on the
 * stream: read them, and outs[j].data, after synchronising that stream.  outs[j].r
 * is not written.  The workspace and the inputs must stay untouched until then;
 * the next call on the context waits for this one.  Argument errors are returned
 * before anything is enqueued; the per-launch profiler must be off.  Planned at the
 * bounds, every left-to-right R factor must have at most 1024 rows at its bound
 * (TT_ENOTIMPL for the call otherwise: use tt_round_batched). */
tt_status tt_round_batched_async(tt_ctx* ctx, int32_t njobs, const tt_sum* xs, const double* deltas,
                                 const int64_t* max_ranks, tt_vec* outs, int32_t* ranks, int32_t* job_status,
                                 double* norms);

/* Graph replay of tt_round_batched_async (for loops that round new data in the same
 * buffers): when on, the first call with a given set of arguments -- every pointer,
 * shape, rank, coefficient, accuracy, rank cap and capacity, the workspace and the
 * result arrays -- runs and is then captured as a HIP graph on the context's stream
 * (which must not be the legacy default stream; there the capture is refused and the
 * calls run directly); later calls with the same arguments launch that graph, which
 * reads whatever the input buffers hold by then.  Each entry keeps its task
 * descriptors in a device block of its own (a few MB); at most 16 entries, the least
 * recently used dropped.  Off (0) drops them all.  tt_ctx_graph_count returns the
 * number of entries that hold a graph. */
tt_status tt_ctx_set_graphs(tt_ctx* ctx, int on);
int32_t tt_ctx_graph_count(const tt_ctx* ctx);

/* Truncated SVD of the left-to-right sweep of TT-round (Section 2): the R factor of each
 * step is diagonalised by one-sided Jacobi, in one workgroup when it has at most `rows`
 * rows and by block Jacobi over many workgroups above (column blocks of 32, one
 * workgroup per pair of blocks in each round).  Both give the singular values to working
 * precision; the crossover is a speed setting.  rows in [32, 1024] (default 224); R
 * factors of more than 4096 rows are not supported (TT_ENOTIMPL).  TT_EINVAL outside. */
tt_status tt_ctx_set_svd_block_min(tt_ctx* ctx, int32_t rows);

/* Upper bound on the packed size (elements) of TT-round(x): ranks are capped
 * by min(sum of component ranks, prod n_{<=k}, prod n_{>k}). */
int64_t tt_round_out_capacity(const tt_sum* x);

/* Accuracy tt_round(x, delta) guarantees: ||x - x~|| <= delta_eff ||x||.  FP64:
 * delta_eff = delta.  FP32-bulk: the per-bond threshold is
 * max(delta / sqrt(d-1), 2 sqrt(s_k) u_32) ||x||, s_k the columns of the merged
 * core at bond k, because singular values below the FP32 resolution of that
 * core are noise (keeping them only inflates the ranks); so delta_eff =
 * max(delta, sqrt(d-1) 2 sqrt(s_max) u_32) with s_max bounded by the summed
 * ranks and the rank caps.  Host-only.  -1 on bad input. */
double tt_round_effective_delta(const tt_sum* x, double delta);

/* Workspace bytes tt_round needs for x (batched: sum over jobs). */
int64_t tt_round_workspace_bytes(const tt_sum* x);

/* Orthogonalize m TT-vectors a[0..m-1] (each a lazy sum) with rounding
 * accuracy delta (Section 3):  TT_CGS Algorithm 1, TT_MGS Algorithm 2,
 * TT_CGS2 Algorithm 3, TT_MGS2 Algorithm 4, TT_GRAM Algorithm 5,
 * TT_HOUSEHOLDER Algorithms 6-8 (Section 3.3: Householder TT-vectors against
 * the canonical basis e_i = e_{i_1} x ... x e_{i_d}, first index fastest; the
 * diagonal of R takes the stable sign, R(i,i) = -sign(<a~_i, e_i>) times the
 * remaining norm; 4m - 1 roundings; m must not exceed prod n_k; the
 * Householder vectors live in the workspace, whose required size the library
 * reports through TT_ECAPACITY before any work starts).
 * Outputs: q[0..m-1] (caller buffers with capacity; r written), R (HOST,
 * m*m column-major, upper triangular, A ~ Q R: column i holds the
 * projections of a_i), loo (HOST [m], nullable: ||I_k - Q_k^T Q_k||_2 for
 * k = 1..m), stats (nullable).  rank_guard > 0 stops with TT_EGUARD when a
 * vector to be rounded would exceed that bond rank; q and the columns of R of
 * the stats->m_reached completed vectors are then valid (TT_HOUSEHOLDER forms
 * every q at the end, so none).  Errors: TT_ENOTSPD (Gram: Cholesky fails),
 * TT_EBREAKDOWN (||p|| = 0; Householder: a~_i in the span of e_0..e_{i-1}). */
tt_status tt_orthogonalize(tt_ctx* ctx, tt_scheme scheme, int32_t m, const tt_sum* a, double delta,
                           int64_t rank_guard, tt_vec* q, double* R, double* loo,
                           tt_ortho_stats* stats);

/* Output capacities of tt_orthogonalize for the m inputs a (Section 3: the ranks
 * of the sum a scheme rounds bound the ranks of its result, and every rank is
 * capped by min(prod n_{<=k}, prod n_{>k}) and by rank_guard when > 0):
 * upper bounds of the bond ranks of each q_i -- CGS/MGS rank(a_i) + sum_{j<i}
 * bound(q_j); CGS2/MGS2 min(that, caps) + sum_{j<i} bound(q_j) (the second pass
 * rounds the first pass's result plus the basis); Gram sum_{k<=i} rank(a_k);
 * Householder 1 + sum_{l<=i} bound(u_l) with bound(u_l) = rank(a_l) +
 * sum_{j<l} bound(u_j) + l + 1.  ranks (HOST [m*(d+1)], nullable) receives the
 * bounds of q_i at ranks[i*(d+1) + k]; sizes (HOST [m], nullable) the packed
 * element counts, i.e. the capacity each q[i] needs.  Host-only: reads only the
 * shapes (the data pointers may be NULL).  Errors: TT_EINVAL. */
tt_status tt_orthogonalize_capacity(int32_t scheme, int32_t m, const tt_sum* a, int64_t rank_guard, int64_t* ranks,
                                    int64_t* sizes);

/* Randomized rounding of a lazy sum (the cheaper rounding of sums that the
 * paper cites for output ranks far below those of the sum):
 * Randomize-then-Orthogonalize with the Gaussian sketch TT-vector `sketch`
 * (ranks l_k, drawn by the caller, same d and n as x): W_k = partial
 * contractions of x and the sketch from the right; from the left, core k of
 * the result is Q of Z_k = L(G_k) W_{k+1} and M_k = Q^T L(G_k) is absorbed into
 * core k+1.  Result ranks min(l_k, p_{k-1} n_k); with delta > 0 the result is
 * then rounded deterministically at delta (as tt_round).  The sketch is FP64;
 * x and out are FP64, or FP32 (the components are converted to FP64 in the
 * workspace, the sweep runs in FP64, its result is converted back and the
 * rounding at delta is FP32-bulk); d = 1 returns the (rounded) sum.  out: device, capacity set
 * by the caller (out->r written).  No QR of the R_k-column unfoldings of the
 * sum is formed, so R_k may exceed the tile limits of tt_round; the sketch
 * ranks must keep Z_k within them.  Works in the context workspace (the
 * sketch contractions, the sketched cores and their QR trees; FP32 inputs add
 * an FP64 copy of the components).  Errors: TT_EINVAL (shapes, an FP32
 * sketch, x and out differing in dtype, delta < 0), TT_ECAPACITY (out or the
 * workspace too small; the required workspace is then reported by
 * tt_ctx_required_bytes), TT_ENOTIMPL (a sketch rank above 1024, or a sketched
 * core beyond the tile limits). */
tt_status tt_round_randomized(tt_ctx* ctx, const tt_sum* x, const tt_vec* sketch, double delta, tt_vec* out);

/* y = alpha * Delta_d x: the discrete Laplacian of order d with Dirichlet
 * boundary conditions (Section 4, the operator of the Krylov inputs) as the
 * rank-two TT-matrix with cores [L, I], [[I, 0], [L, I]], [I; L], where
 * L = (n_k + 1)^2 tridiag(1, -2, 1) on mode k.  out (device, capacity set by
 * the caller, no aliasing with x) receives ranks r_0 = r_d = 1 and 2 r_k in
 * between (rank 1 when d = 1); alpha goes on the first core.  Errors:
 * TT_EINVAL (shapes, non-finite alpha, aliasing), TT_ECAPACITY. */
tt_status tt_laplacian(tt_ctx* ctx, const tt_vec* x, double alpha, tt_vec* out);

/* The m input vectors of the experiments of Section 4: x_1 is the TT-vector
 * of ones; a_j is x_j rounded with the accuracy replaced by the rank cap one
 * and normalised; x_{j+1} = -Delta_d a_j.  a[0..m-1]: device outputs of one
 * shape (d, n, dtype taken from a[0]), capacity >= sum_k n_k each; their ranks
 * are written (all 1).  Works in the context workspace (4 sum_k n_k elements
 * plus one rounding).  Errors: TT_EINVAL, TT_ECAPACITY, TT_EBREAKDOWN. */
tt_status tt_krylov_laplacian(tt_ctx* ctx, int32_t m, tt_vec* a);

/* Loss of orthogonality ||I_k - Q_k^T Q_k||_2, k = 1..m (Section 3.4):
 * Gram matrix of q by TT inner products, then the largest |eigenvalue| of
 * each leading block (symmetric Jacobi on the device).  loo: HOST [m];
 * gram (HOST m*m, nullable) receives Q^T Q. */
tt_status tt_loo(tt_ctx* ctx, int32_t m, const tt_vec* q, double* loo, double* gram);

/* Condition numbers kappa(A_k) = sigma_max / sigma_min of A_k = [a_0 .. a_{k-1}],
 * k = 1..m, for m lazy sums of one shape (the conditioning against which
 * Section 3.4 bounds the loss of orthogonality of each scheme and Section 4
 * plots it): the FP64 Gram matrix G(i, j) = <a_i, a_j> by TT inner products
 * (FP64 accumulation for either dtype), then kappa(A_k) = sqrt(kappa(G_k)) from
 * the singular values of each leading block (symmetric Jacobi on the device).
 * Meaningful while kappa(G_k) stays well below 1 / u_64, i.e. kappa(A_k) below
 * about 1e7; beyond that the smallest eigenvalue of G_k is rounding noise.
 * kappa: HOST [m] (INFINITY where G_k is singular to working precision); gram:
 * HOST m*m row-major or NULL.  Errors: TT_EINVAL (shapes), TT_ECAPACITY. */
tt_status tt_cond(tt_ctx* ctx, int32_t m, const tt_sum* a, double* kappa, double* gram);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): <x, y> of two TT-vectors x and y
 * (same d, n and dtype; plain TT-vectors, not lazy sums) with the contraction
 * of tt_dot (FP64 products and sums for either dtype), written to the DEVICE
 * double *out.  No context: one kernel launch on `stream` (a hipStream_t of the
 * current device, NULL for the default stream); the call neither allocates
 * nor synchronises, so *out is valid once the stream reaches that point.
 * Scratch: a fixed 16 MiB device array inside the library, one per device,
 * held from the first call on that device until the process ends; a pair needs
 * (2 max_k rx_k ry_k rounded up to 32) + max_k rx_k n_k ry_{k+1} doubles of it.
 * Every call on a device shares that device's array, so calls that overlap on
 * one device (other streams, other threads) race; calls ordered on one stream
 * do not.  Errors: TT_EINVAL (shapes, null pointers, capacity below the packed
 * size), TT_ECAPACITY (the pair needs more than the 16 MiB), TT_EDEVICE. */
tt_status tt_dot_noalloc(void* stream, const tt_vec* x, const tt_vec* y, double* out);

/* ---------------------------------------------------------------------------
 * Serving engine: continuous batching of orthogonalization requests.
 *
 * A request orthogonalizes one new TT-vector w (a lazy sum) against an
 * orthonormal basis q_0..q_{b-1} that stays resident on the device (the
 * Krylov basis of a TT-GMRES solver): one step i = b of TT-CGS (Algorithm 1),
 * TT-MGS (Algorithm 2), TT-CGS2 (Algorithm 3) or TT-MGS2 (Algorithm 4).
 * Every tt_engine_step advances each request in flight by one stage -- the
 * batched inner products and projection coefficients of a pass, the
 * rounding of a pass, or the final normalisation -- and all requests at the
 * same kind of stage share the same launches.  Requests submitted between
 * steps join the next step while older ones are still in flight.  A
 * request's results do not depend on the other requests in flight.
 * ------------------------------------------------------------------------- */
typedef struct tt_request {
  int32_t scheme;             /* TT_CGS, TT_MGS, TT_CGS2 or TT_MGS2                         */
  int32_t b;                  /* basis size >= 0                                           */
  const tt_vec* basis;        /* [b] orthonormal basis (device data, not modified)         */
  const double* basis_gram;   /* HOST b*b row-major <q_l, q_j>, used by the MGS schemes;
                                 NULL means the identity                                    */
  tt_sum w;                   /* the new vector                                           */
  double delta;               /* rounding accuracy                                        */
  tt_vec* q_out;              /* result q_b = p / ||p|| (capacity >= tt_request_out_capacity) */
  double* r_out;              /* HOST [b + 1]: column b of R (projections, then ||p||)    */
  double* gram_out;           /* HOST [b] or NULL: <q_b, q_j>, j < b (next basis Gram row) */
  void* scratch;              /* device memory of tt_request_scratch_bytes bytes,
                                 owned by the caller until the request completes           */
  int64_t scratch_bytes;
} tt_request;

typedef struct tt_engine tt_engine;

/* Element capacity q_out needs, and device scratch bytes a request needs
 * (the basis Gram, the first-pass vector of CGS2/MGS2).  -1 on bad input. */
int64_t tt_request_out_capacity(const tt_request* r);
int64_t tt_request_scratch_bytes(const tt_request* r);

/* An engine works on the context's stream and workspace; one host thread. */
tt_status tt_engine_create(tt_ctx* ctx, tt_engine** e);
void tt_engine_destroy(tt_engine* e);
/* Validate and enqueue a request (copied; the pointed-to buffers must stay
 * valid until it completes).  *id identifies it in tt_engine_step. */
tt_status tt_engine_submit(tt_engine* e, const tt_request* r, int64_t* id);
/* Advance every request in flight by one stage.  Up to max_done completed
 * requests are reported in done_ids / done_status (HOST arrays); *ndone
 * receives their number.  A failed request (TT_EBREAKDOWN when ||p|| = 0,
 * TT_ECAPACITY, TT_ENOTIMPL for unsupported shapes) is reported with its
 * status; the others continue.  The return value is TT_OK unless the engine
 * itself failed (device error). */
tt_status tt_engine_step(tt_engine* e, int32_t max_done, int64_t* done_ids, tt_status* done_status,
                         int32_t* ndone);
/* Requests submitted and not yet reported. */
int32_t tt_engine_pending(const tt_engine* e);

#ifdef __cplusplus
}
#endif
#endif /* TTORTHO_H */
