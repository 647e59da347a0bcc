// Host-side internals of the C ABI: context, allocators, TSQR planning and the
// batched TT-round pipeline.  Only host code lives here; every arithmetic step
// of the method runs in the kernels declared in common.h.
#pragma once
#include <cmath>
#include <cstring>
#include <string>
#include <memory>
#include <vector>

#include "../../include/ttortho.h"
#include "common.h"

namespace tto {

// Library-owned growable arena (device or pinned host) for task descriptors
// and small scalars.  Chunks allocated during a call stay valid until reset().
struct Arena {
  bool pinned = false;
  std::vector<std::pair<char*, size_t>> chunks;
  size_t off = 0;
  size_t used_total = 0;
  char* alloc(size_t bytes);
  void reset();
  void release();
};

// Device block of a captured graph: descriptors and small scalars of one call,
// allocated in the same order on every pass, so that after rewind() the same
// request sequence yields the same addresses (the capture pass then finds the
// descriptors the first pass uploaded already in place).
struct ReplayArena {
  std::vector<std::pair<char*, size_t>> chunks;
  size_t cur = 0, off = 0;
  char* alloc(size_t bytes);
  void rewind() {
    cur = 0;
    off = 0;
  }
  void release();
};

// A captured tt_round_batched_async call: the exact argument bytes it was taken
// for, its descriptor block and the instantiated graph (null: not capturable).
struct GraphEntry {
  std::string sig;
  ReplayArena arena;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

}  // namespace tto

namespace tto {
// Kinds of launches timed by the context's profiler.
enum ProfKind { PK_QR_LEAF = 0, PK_QR_NODE, PK_QR_APPLY, PK_SVD, PK_GEMM, PK_DOT, PK_OTHER, PK_COUNT };
struct ProfRec {
  int kind;
  hipEvent_t start, stop;
  double flops;
  double bytes;
};
}  // namespace tto

struct tt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;  // second stream (default priority) for work off the critical path
  hipStream_t upload_stream = nullptr;   // stream of task-descriptor uploads (null: stream)
  std::vector<hipEvent_t> ev_pool;   // timing-free events for stream dependencies
  size_t ev_used = 0;
  char* ws = nullptr;          // caller workspace
  size_t ws_bytes = 0;
  size_t ws_off = 0;
  bool ws_overflow = false;
  size_t required = 0;
  tto::Arena dev;              // task descriptors, scalars
  tto::Arena pin;              // staging for uploads / readbacks
  std::string err;
  // profiler: HIP events around each launch on this context's stream
  bool prof = false;
  bool autotune = false;       // time candidate TSQR tree shapes for unseen shapes
  hipEvent_t async_done = nullptr;   // end of the last asynchronous call on this context
  bool async_pending = false;        // the next call waits for it before reusing any buffer
  // graph replay of repeated asynchronous batched roundings
  bool graphs = false;
  std::vector<tto::GraphEntry*> graph_cache;
  uint64_t graph_clock = 0;
  tto::ReplayArena* graph_arena = nullptr;   // set while a call builds or captures an entry
  bool graph_capturing = false;              // uploads find their data in place: no copies
  uint64_t tune_count = 0;                   // tree-shape tunings run (they allocate and launch too)
  int svd_block_min = tto::SVD_BLOCK_MIN;    // R factors of more rows take the block Jacobi SVD
  std::vector<tto::ProfRec> prof_open;
  std::vector<hipEvent_t> prof_pool;
  double prof_ms[tto::PK_COUNT] = {0};
  double prof_flops[tto::PK_COUNT] = {0};
  double prof_bytes[tto::PK_COUNT] = {0};
  int64_t prof_cnt[tto::PK_COUNT] = {0};
};

namespace tto {

// ---- helpers used by the API implementation -------------------------------
tt_status fail(tt_ctx* c, tt_status s, const std::string& msg);
tt_status hip_fail(tt_ctx* c, hipError_t e, const char* where);

// bump allocation in the caller workspace (256-byte aligned).  On overflow
// returns nullptr and records the needed size; callers check c->ws_overflow
// before launching anything.
void* ws_alloc(tt_ctx* c, size_t bytes);

template <typename T>
T* ws_alloc_n(tt_ctx* c, size_t n) {
  return (T*)ws_alloc(c, n * sizeof(T));
}

// upload a host array to a library-owned device buffer (stream ordered)
void* upload_bytes(tt_ctx* c, const void* src, size_t bytes);
template <typename T>
T* upload(tt_ctx* c, const std::vector<T>& v) {
  if (v.empty()) return nullptr;
  return (T*)upload_bytes(c, v.data(), v.size() * sizeof(T));
}
// two host arrays in one upload (one copy on the stream); b starts at a 256-byte boundary
template <typename A, typename B>
bool upload_pair(tt_ctx* c, const std::vector<A>& a, const std::vector<B>& b, const A** da, const B** db) {
  *da = nullptr;
  *db = nullptr;
  if (a.empty() && b.empty()) return true;
  const size_t na = a.size() * sizeof(A), off = (na + 255) & ~(size_t)255, nb = b.size() * sizeof(B);
  std::vector<char> h(off + nb);
  if (na) std::memcpy(h.data(), a.data(), na);
  if (nb) std::memcpy(h.data() + off, b.data(), nb);
  char* d = (char*)upload_bytes(c, h.data(), h.size());
  if (!d) return false;
  *da = a.empty() ? nullptr : (const A*)d;
  *db = b.empty() ? nullptr : (const B*)(d + off);
  return true;
}
void* dev_scratch(tt_ctx* c, size_t bytes);

inline size_t elt_size(int dtype) { return dtype == TT_F64 ? 8 : 4; }

// Profiler: prof_begin before a launch, prof_end after it (no-ops when off);
// prof_collect after the stream has drained accumulates the elapsed times.
int prof_begin(tt_ctx* c, int kind, double flops, double bytes, hipStream_t s = nullptr);
void prof_end(tt_ctx* c, int rec, hipStream_t s = nullptr);

// Side stream of the context (created on first use) and a dependency event
// (recycled when the call ends).  Both streams are drained by every entry point.
hipStream_t side_stream(tt_ctx* c);
hipEvent_t dep_event(tt_ctx* c);
void prof_collect(tt_ctx* c);

// ---- TSQR tree -------------------------------------------------------------
struct Tree {
  int64_t M = 0, N = 0;
  int leaf_dtype = 0;                           // 0 f64, 1 f32
  std::vector<std::vector<QrTask>> lvl;         // lvl[0] = leaves
  std::vector<int64_t> leaf_row0;               // first row of each leaf
  // Column-blocked QR, for a matrix too wide for one tree (more than QR_MAXROWS rows and
  // more than QR_MAXROWS / 2 columns): the tiles factor the first nf columns and carry
  // the others through their reflectors; the rows each tile leaves behind (rows
  // min(m, nf)..m-1 of the carried columns, tiles in level order) are gathered into
  // `rest`, (M - nf) x (N - nf) in the leaf dtype, which `next` factors in turn.  Then
  // A = Q_1 diag(I, Q_next) [R_11 R_12; 0 R_next] with rows in that gathered order, and
  // R is assembled in rfull (kr x N doubles, ld N).
  // The tiles of a block hold every remaining column only while the block is factored: they
  // live in one region that every block of the chain reuses, and once a block is done each
  // tile's factored columns (the reflectors and R, m x nf) move to `ctile`, which the
  // application of Q reads.  The blocks of a chain share one `rest` buffer, and a nested
  // block writes its R in place inside the outer block's rfull (ld r_ld).
  int64_t nf = 0;                               // 0: an ordinary tree
  std::shared_ptr<Tree> next;
  void* rest = nullptr;
  double* rfull = nullptr;
  int64_t r_ld = 0;
  std::vector<std::vector<void*>> ctile;        // [level][tile]: m x nf, ld nf
  int kr() const;                               // rows of the R factor
  const void* root_R() const;                   // R (row-major, ld = rld(); entries left of the diagonal not read)
  int64_t rld() const { return next ? r_ld : N; }
  int root_f32() const { return !next && lvl.size() == 1 && leaf_dtype == TT_F32 ? 1 : 0; }   // dtype of root_R
  int depth() const { return (int)lvl.size(); }
  int64_t fk() const { return next ? nf : N; }  // columns the tiles factor
};

// Plan (and carve from `alloc`) a TSQR tree for an M x N matrix whose element
// (r, c) is at src[r*rs + c*cs] (dtype of the leaves).  Returns false when the
// shape is outside what the tile kernels support.
struct Carver {
  tt_ctx* ctx = nullptr;    // carve from workspace when base == nullptr
  char* base = nullptr;     // carve inside a reserved block
  size_t off = 0, cap = 0;
  bool measure = false;
  void* take(size_t bytes);
};
bool plan_tree(Carver& cv, Tree& t, int64_t M, int64_t N, int dtype, const void* src, int64_t rs, int64_t cs,
               std::string* why);

// TSQR tree shape: rows of a leaf tile and children per tree node.  The
// autotuner times candidate shapes on synthetic data once per (dtype, N,
// ceil(log2 M)) and records the fastest; plan_tree uses a recorded shape when
// there is one, else default_shape.
struct TreeShape {
  int32_t leaf_rows;
  int32_t fanin;
};
TreeShape default_shape(int64_t M, int64_t N);
bool tuned_shape(int64_t M, int64_t N, int dtype, TreeShape* out);
void set_tuned_shape(int64_t M, int64_t N, int dtype, TreeShape sh);
tt_status tune_tree(tt_ctx* c, int64_t M, int64_t N, int dtype, TreeShape* best);

// ---- rounding jobs ---------------------------------------------------------
struct Comp {
  const char* data = nullptr;
  int64_t r[TT_MAXD + 1];
  int64_t core_off[TT_MAXD];
  double coef = 1.0;
};

struct RJob {
  int d = 0;
  int dtype = 0;
  int64_t n[TT_MAXD];
  std::vector<Comp> comps;
  std::vector<int64_t> roff;      // [ncomp * (d+1)] rank offset of each component per bond
  int64_t R[TT_MAXD + 1];         // summed ranks
  double delta = 0.0;
  int64_t max_rank = 0;
  tt_vec* out = nullptr;
  double norm = 0.0;
  tt_status status = TT_OK;
  bool orth_only = false;         // right-to-left sweep and norm only (no output TT)
};

tt_status make_job(tt_ctx* c, const tt_sum* x, double delta, int64_t max_rank, tt_vec* out, RJob& job);
// How a batch of roundings is sequenced.  By default the host reads the rank the
// device chose after every left-to-right step and plans the next step at that
// rank.  With bound_plan every step is planned at the rank bounds (the data
// beyond the chosen rank is zero), the cores are formed at their bound shapes in
// a staging area and compacted on the device at the end, so nothing waits for the
// host until the final read-back; with async even that read-back is left to
// copies into the caller's pinned arrays and the call returns once everything
// is enqueued.
struct RoundMode {
  bool bound_plan = false;
  bool async = false;
  int32_t* ranks = nullptr;    // async: caller pinned [njobs * (TT_MAXD + 1)]
  int32_t* status = nullptr;   // async: caller pinned [njobs]
  double* norms = nullptr;     // async: caller pinned [njobs] or null
};
tt_status round_jobs(tt_ctx* c, std::vector<RJob>& jobs, const RoundMode& mode = RoundMode());
int64_t round_workspace_bytes(const std::vector<RJob>& jobs);
// round_jobs on consecutive groups of the jobs whose workspaces together stay within the
// largest single job's (or 32 GiB): one batch for moderate jobs, memory bounded by the
// largest job for large ones (the schemes' batched final roundings)
tt_status round_jobs_grouped(tt_ctx* c, std::vector<RJob>& jobs);
// FP32-bulk noise floor of the per-bond threshold, relative to ||x||, for a
// merged core with s columns: 2 sqrt(s) u_32 (the level below which the SVD
// sets columns aside as unresolved in FP32).
inline double fp32_eps_floor(int64_t s) { return 2.0 * std::sqrt((double)(s > 1 ? s : 1)) * 5.9604644775390625e-08; }
// Randomize-then-Orthogonalize rounding of a lazy FP64 sum with the sketch TT
// sk (ranks l_k); with delta > 0 the result is then rounded deterministically.
tt_status round_randomized(tt_ctx* c, const tt_sum* x, const tt_vec* sk, double delta, tt_vec* out);

// ---- inner products ----------------------------------------------------------
// out_dev[p] = <xs[p], ys[p]> (device doubles)
tt_status dot_pairs(tt_ctx* c, int npairs, const tt_sum* xs, const tt_sum* ys, double* out_dev);

}  // namespace tto
