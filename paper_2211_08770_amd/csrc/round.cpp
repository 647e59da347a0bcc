// Batched TT-round (Section 2 of the paper; the two-sweep rounding it cites).
//
// All jobs of a batch advance in lock step: every launch gathers the tasks
// of all jobs that are at the same step, so uneven jobs (different order,
// mode sizes, ranks and number of sum components) share launches.
//
//   right-to-left, core k = d-1..1:
//     Y_k   = column-major view (n_k s_{k+1}) x R_k of the current core k
//     Y_k   = Q_k R_k      (TSQR: Householder tiles, FP64 tree, Q_k kept implicit)
//     core k-1 <- core k-1 x_3 R_k^T   (block-aware GEMM per sum component)
//   ||x|| = ||G_0||_F ;  eps = delta / sqrt(d-1) * ||x||
//   left-to-right, core k = 0..d-2:
//     C_k   = W_k x_1 Q_k-core            (apply Q_k to [W_k^T; 0])
//     L(C_k) = Q_M R_M                    (TSQR)
//     R_M   = U S V^T                     (FP64 one-sided Jacobi; rank t_{k+1} on device)
//     core k of the result = Q_M [U_t; 0] ; W_{k+1} = S_t V_t^T
//   last core = W_{d-1} x_1 Q_{d-1}-core
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "host.h"

namespace tto {

namespace {

int npanels(int64_t k) { return (int)((k + QR_NB - 1) / QR_NB); }

}  // namespace

// ---- tree shapes picked by the autotuner (process-wide: a property of the
// device and the shape, shared by every context so that workspace sizing and
// planning always agree)
namespace {
std::mutex g_tune_mu;
std::map<uint64_t, TreeShape> g_tune;
}  // namespace

uint64_t tune_key(int64_t M, int64_t N, int dtype) {
  int lb = 0;
  while (lb < 62 && (int64_t(1) << lb) < M) ++lb;
  return (uint64_t)(dtype & 1) | ((uint64_t)N << 1) | ((uint64_t)lb << 40);
}

bool tuned_shape(int64_t M, int64_t N, int dtype, TreeShape* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tune_key(M, N, dtype));
  if (it == g_tune.end()) return false;
  if (out) *out = it->second;
  return true;
}

void set_tuned_shape(int64_t M, int64_t N, int dtype, TreeShape sh) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[tune_key(M, N, dtype)] = sh;
}

TreeShape default_shape(int64_t M, int64_t N) {
  TreeShape sh;
  sh.leaf_rows = (int32_t)(M <= QR_MAXROWS ? M : std::min<int64_t>(QR_MAXROWS, std::max<int64_t>(2 * N, 64)));
  sh.fanin = (int32_t)std::max<int64_t>(2, QR_MAXROWS / std::max<int64_t>(N, 1));
  return sh;
}

void* Carver::take(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (base == nullptr && !measure) return ws_alloc(ctx, bytes);
  void* p = measure ? nullptr : base + off;
  off += bytes;
  if (!measure && off > cap) return nullptr;
  return p;
}

int Tree::kr() const {
  if (next) return (int)(nf + next->kr());
  const QrTask& r = lvl.back()[0];
  return (int)std::min<int64_t>(r.m, N);
}

const void* Tree::root_R() const { return next ? (const void*)rfull : lvl.back()[0].tile; }

bool plan_tree_shape(Carver& cv, Tree& t, int64_t M, int64_t N, int dtype, const void* src, int64_t rs, int64_t cs,
                     TreeShape sh, std::string* why);

bool plan_tree(Carver& cv, Tree& t, int64_t M, int64_t N, int dtype, const void* src, int64_t rs, int64_t cs,
               std::string* why) {
  TreeShape sh = default_shape(M, N);
  TreeShape tuned;
  if (tuned_shape(M, N, dtype, &tuned)) sh = tuned;
  return plan_tree_shape(cv, t, M, N, dtype, src, rs, cs, sh, why);
}

// The region the full-width tiles of a chain of column blocks share.
struct WideArea {
  char* base = nullptr;
  size_t cap = 0;
  bool measure = false;
};

static bool plan_tree_impl(Carver& cv, Tree& t, int64_t M, int64_t N, int dtype, const void* src, int64_t rs,
                           int64_t cs, TreeShape req, std::string* why, const WideArea* wide, void* shared_rest,
                           double* rfull_in, int64_t r_ld_in);

bool plan_tree_shape(Carver& cv, Tree& t, int64_t M, int64_t N, int dtype, const void* src, int64_t rs, int64_t cs,
                     TreeShape req, std::string* why) {
  return plan_tree_impl(cv, t, M, N, dtype, src, rs, cs, req, why, nullptr, nullptr, nullptr, 0);
}

static bool plan_tree_impl(Carver& cv, Tree& t, int64_t M, int64_t N, int dtype, const void* src, int64_t rs,
                           int64_t cs, TreeShape req, std::string* why, const WideArea* wide, void* shared_rest,
                           double* rfull_in, int64_t r_ld_in) {
  t.M = M;
  t.N = N;
  t.leaf_dtype = dtype;
  t.lvl.clear();
  t.leaf_row0.clear();
  t.nf = 0;
  t.next.reset();
  t.rest = nullptr;
  t.rfull = nullptr;
  t.r_ld = 0;
  t.ctile.clear();
  if (M < 1 || N < 1) {
    if (why) *why = "empty QR shape";
    return false;
  }
  const size_t elt = elt_size(dtype);
  // a requested shape must keep every tile within the LDS panel: leaves of
  // at least min(N, M) rows, nodes of at most QR_MAXROWS stacked rows
  TreeShape sh = default_shape(M, N);
  if (req.leaf_rows >= std::min<int64_t>(N, M) && req.leaf_rows <= QR_MAXROWS && req.fanin >= 2 &&
      (int64_t)req.fanin * std::min<int64_t>(req.leaf_rows, N) <= QR_MAXROWS)
    sh = req;
  int64_t b, g = sh.fanin, fk = N;   // leaf rows, fan-in, columns the tiles factor
  if (M <= QR_MAXROWS && sh.leaf_rows >= M) {
    b = M;
  } else if (N > QR_MAXROWS / 2) {
    // too wide for one tree: the first column block, its trailing rows factored by `next`
    fk = QR_BLOCK_COLS;
    b = 2 * fk;
    g = 2;
  } else {
    b = sh.leaf_rows;
  }
  const int32_t nfact = fk < N ? (int32_t)fk : 0;
  const int64_t nleaves = (M + b - 1) / b;
  std::vector<QrTask> leaves;
  leaves.reserve(nleaves);
  for (int64_t j = 0; j < nleaves; ++j) {
    const int64_t r0 = j * b;
    const int64_t m = std::min<int64_t>(b, M - r0);
    const int64_t k = std::min<int64_t>(m, fk);
    QrTask q;
    std::memset(&q, 0, sizeof(q));
    q.src = src ? (const char*)src + (size_t)(r0 * rs) * elt : nullptr;
    q.src_rs = rs;
    q.src_cs = cs;
    q.m = (int32_t)m;
    q.ncol = (int32_t)N;
    q.nfact = nfact;
    if (!nfact) q.tile = cv.take((size_t)m * N * elt);   // (column blocks: below)
    q.tau = (double*)cv.take((size_t)k * 8);
    q.tmat = cv.take((size_t)npanels(k) * QR_NB * QR_NB * 8);
    leaves.push_back(q);
    t.leaf_row0.push_back(r0);
  }
  t.lvl.push_back(std::move(leaves));
  while (t.lvl.back().size() > 1) {
    const std::vector<QrTask>& prev = t.lvl.back();
    std::vector<QrTask> nodes;
    for (size_t i = 0; i < prev.size(); i += (size_t)g) {
      const int cnt = (int)std::min<size_t>((size_t)g, prev.size() - i);
      int64_t rows = 0;
      for (int c = 0; c < cnt; ++c) rows += std::min<int64_t>(prev[i + c].m, fk);
      const int64_t k = std::min<int64_t>(rows, fk);
      QrTask q;
      std::memset(&q, 0, sizeof(q));
      q.nchild = cnt;
      q.child0 = (int32_t)i;
      // every child but the last contributes the same number of R rows (the kernels rely on it)
      q.kc0 = (int32_t)std::min<int64_t>(prev[i].m, fk);
      q.kc_last = (int32_t)std::min<int64_t>(prev[i + cnt - 1].m, fk);
      for (int c = 0; c + 1 < cnt; ++c)
        if (std::min<int64_t>(prev[i + c].m, fk) != q.kc0) {
          if (why) *why = "internal: uneven TSQR children";
          return false;
        }
      q.m = (int32_t)rows;
      q.ncol = (int32_t)N;
      q.nfact = nfact;
      if (!nfact) q.tile = cv.take((size_t)rows * N * 8);
      q.tau = (double*)cv.take((size_t)k * 8);
      q.tmat = cv.take((size_t)npanels(k) * QR_NB * QR_NB * 8);
      nodes.push_back(q);
    }
    t.lvl.push_back(std::move(nodes));
  }
  if (nfact) {
    // full-width tiles in the chain's shared region (the first block of a chain sizes it: the
    // later blocks have fewer rows and columns), the factored columns of each tile kept apart
    auto full_bytes = [&](size_t l, const QrTask& q) {
      return (((size_t)q.m * N * (l == 0 ? elt : 8)) + 255) & ~(size_t)255;
    };
    WideArea wa;
    if (wide) {
      wa = *wide;
    } else {
      size_t need = 0;
      for (size_t l = 0; l < t.lvl.size(); ++l)
        for (const QrTask& q : t.lvl[l]) need += full_bytes(l, q);
      wa.base = (char*)cv.take(need);
      wa.cap = need;
      wa.measure = cv.measure || wa.base == nullptr;
    }
    Carver wcv;
    wcv.base = wa.base;
    wcv.cap = wa.cap;
    wcv.measure = wa.measure;
    t.ctile.resize(t.lvl.size());
    for (size_t l = 0; l < t.lvl.size(); ++l)
      for (QrTask& q : t.lvl[l]) {
        q.tile = wcv.take(full_bytes(l, q));
        t.ctile[l].push_back(cv.take((size_t)q.m * fk * (l == 0 ? elt : 8)));
      }
    if (!wcv.measure && wcv.off > wcv.cap) {
      if (why) *why = "internal: column-block tiles exceed their region";
      return false;
    }
    // the trailing block: rows left behind by the tiles, in level order, factored by an
    // ordinary (or again blocked) tree of the default shape
    t.nf = fk;
    t.rest = shared_rest ? shared_rest : cv.take((size_t)(M - fk) * (N - fk) * elt);
    if (wide) {   // a nested block writes its R inside the outer block's
      t.rfull = rfull_in;
      t.r_ld = r_ld_in;
    } else {
      t.rfull = (double*)cv.take((size_t)std::min(M, N) * N * 8);
      t.r_ld = N;
    }
    t.next = std::make_shared<Tree>();
    double* inner_r = t.rfull ? t.rfull + fk * t.r_ld + fk : nullptr;
    if (!plan_tree_impl(cv, *t.next, M - fk, N - fk, dtype, t.rest, N - fk, 1, default_shape(M - fk, N - fk), why,
                        &wa, t.rest, inner_r, t.r_ld))
      return false;
  }
  return true;
}

// First row of each tile's left-behind rows (rows min(m, nf)..m-1) in the trailing
// block of a column-blocked tree: tiles in level order, leaves first.
static std::vector<std::vector<int64_t>> rest_offsets(const Tree& t) {
  std::vector<std::vector<int64_t>> off(t.lvl.size());
  int64_t o = 0;
  for (size_t l = 0; l < t.lvl.size(); ++l)
    for (const QrTask& q : t.lvl[l]) {
      off[l].push_back(o);
      o += q.m - std::min<int64_t>(q.m, t.nf);
    }
  return off;
}

namespace {

// rows of column j that the Householder reflector of column j touches
int64_t active_rows(int64_t m, int nchild, int64_t kc0, int64_t kc_last, int64_t j) {
  if (nchild == 0) return m - j;
  int64_t a = 0;
  for (int b = 0; b < nchild; ++b) {
    const int64_t off = (int64_t)b * kc0;
    const int64_t kcb = (b == nchild - 1) ? kc_last : kc0;
    const int64_t lo = std::max<int64_t>(0, j - off), hi = std::min<int64_t>(kcb - 1, j);
    if (hi >= lo) a += hi - lo + 1;
  }
  return a;
}

// algorithmic flops of a Householder QR of one tile: sum_j (4 a_j (N-j-1) + 3 a_j)
double qr_flops(const QrTask& q) {
  const int64_t nf = q.nfact > 0 ? q.nfact : q.ncol;   // carried columns are counted with the update
  const int64_t kq = std::min<int64_t>(q.m, nf);
  double f = 0.0;
  for (int64_t j = 0; j < kq; ++j) {
    const double a = (double)active_rows(q.m, q.nchild, q.kc0, q.kc_last, j);
    f += 4.0 * a * (double)(nf - j - 1) + 3.0 * a;
  }
  return f;
}

// algorithmic flops of applying the tile's reflectors to t columns: sum_j 4 a_j t
double apply_flops(const ApplyTask& t) {
  double f = 0.0;
  for (int64_t j = 0; j < t.kq; ++j) f += 4.0 * (double)active_rows(t.m, t.nchild, t.kc0, t.kc_last, j) * t.t;
  return f;
}

// Apply plan of a tree: out = Q [X; 0], tasks grouped top-down.
struct ApplyLevel {
  int tile_dtype;
  std::vector<ApplyTask> tasks;
};

// Scratch of an apply plan: one m x tcols double block per tree node (a node's result is
// its children's input); leaves write straight to the output.
size_t apply_work_bytes(const Tree& t, int64_t tcols) {
  size_t s = 0;
  for (size_t l = 1; l < t.lvl.size(); ++l)
    for (const auto& q : t.lvl[l]) s += (((size_t)q.m * tcols * 8) + 255) & ~(size_t)255;
  if (t.next) s += ((((size_t)(t.M - t.nf) * tcols * 8) + 255) & ~(size_t)255) + apply_work_bytes(*t.next, tcols);
  return s;
}

// Column-blocked tree: Q [X_1; X_2; 0] = Q_1 [X_1; Q_next [X_2; 0]], so the plan of
// `next` (its result Y, in the gathered row order, as double) comes first and every
// tile of the first block then takes its left-behind rows from Y.
void plan_apply(Carver& cv, const Tree& t, const double* X, int64_t x_ld, int64_t tcols, void* out,
                int out_dtype, int64_t out_rs, int64_t out_cs, std::vector<ApplyLevel>& plan) {
  const int L = (int)t.lvl.size();
  const int64_t N = t.fk();
  plan.clear();
  double* Y = nullptr;
  std::vector<std::vector<int64_t>> roff;
  if (t.next) {
    Y = (double*)cv.take((size_t)(t.M - t.nf) * tcols * 8);
    plan_apply(cv, *t.next, X ? X + t.nf * x_ld : nullptr, x_ld, tcols, Y, TT_F64, tcols, 1, plan);
    for (auto& lv : plan)
      for (auto& a : lv.tasks)
        if (a.to_out) a.to_out = 2;   // Y is double whatever the final output's dtype
    roff = rest_offsets(t);
  }
  std::vector<std::vector<double*>> work(L);
  for (int l = 0; l < L; ++l)
    for (size_t i = 0; i < t.lvl[l].size(); ++i)
      work[l].push_back(l == 0 ? nullptr : (double*)cv.take((size_t)t.lvl[l][i].m * tcols * 8));
  // parent of each task and its row offset inside the parent
  std::vector<std::vector<std::pair<int, int64_t>>> parent(L);
  for (int l = 0; l + 1 < L; ++l) {
    parent[l].assign(t.lvl[l].size(), {0, 0});
    for (size_t p = 0; p < t.lvl[l + 1].size(); ++p) {
      const QrTask& nd = t.lvl[l + 1][p];
      int64_t off = 0;
      for (int c = 0; c < nd.nchild; ++c) {
        parent[l][nd.child0 + c] = {(int)p, off};
        off += std::min<int64_t>(t.lvl[l][nd.child0 + c].m, N);
      }
    }
  }
  for (int l = L - 1; l >= 0; --l) {
    ApplyLevel al;
    al.tile_dtype = (l == 0) ? t.leaf_dtype : TT_F64;
    for (size_t i = 0; i < t.lvl[l].size(); ++i) {
      const QrTask& q = t.lvl[l][i];
      ApplyTask a;
      std::memset(&a, 0, sizeof(a));
      a.tile = t.next ? t.ctile[l][i] : q.tile;   // a column block's compact tile: m x nf
      a.tau = q.tau;
      a.tmat = q.tmat;
      a.m = q.m;
      a.ncol = t.next ? (int32_t)t.nf : q.ncol;
      a.kq = (int32_t)std::min<int64_t>(q.m, N);
      a.nchild = q.nchild;
      a.kc0 = q.kc0;
      a.kc_last = q.kc_last;
      a.t = (int32_t)tcols;
      a.work = work[l][i];
      if (Y && q.m > std::min<int64_t>(q.m, N)) {
        a.rest = Y + roff[l][i] * tcols;
        a.rest_ld = tcols;
      }
      if (l == L - 1) {
        a.x = X;
        a.x_ld = x_ld;
        a.k_in = (int32_t)std::min<int64_t>(q.m, N);
      } else {
        const auto& pr = parent[l][i];
        a.x = work[l + 1][pr.first] + pr.second * tcols;
        a.x_ld = tcols;
        a.k_in = (int32_t)std::min<int64_t>(q.m, N);
      }
      if (l == 0) {
        a.to_out = 1;
        a.out = out ? (char*)out + (size_t)(t.leaf_row0[i] * out_rs) * elt_size(out_dtype) : nullptr;
        a.out_rs = out_rs;
        a.out_cs = out_cs;
      }
      al.tasks.push_back(a);
    }
    plan.push_back(std::move(al));
  }
}

struct JobState {
  int64_t s[TT_MAXD + 1];    // right-to-left ranks
  int64_t tb[TT_MAXD + 1];   // bounds of the truncated ranks
  int64_t t[TT_MAXD + 1];    // truncated ranks
  void* Y[TT_MAXD];
  Tree rl[TT_MAXD];
  void* C = nullptr;
  size_t lr_cap = 0;
  char* ap_block = nullptr;
  size_t ap_cap = 0;
  // left-to-right trees and U factors, double-buffered by step parity: the output core of
  // step k is formed on the side stream while step k+1 runs
  Tree lr[2];
  char* lr_blk[2] = {nullptr, nullptr};
  double* urb[2] = {nullptr, nullptr};
  char* ap_side = nullptr;
  double *A = nullptr, *acc = nullptr, *sig = nullptr, *wt = nullptr;
  int32_t* perm = nullptr;
  int32_t* iscr = nullptr;
  double* d_norm = nullptr;
  int64_t out_off = 0;
  bool alive = true;
  // explicit orthogonal factors Q_k (row-major (n_k s_{k+1}) x R_k) of the right-to-left
  // trees, formed on the side stream while the sweep goes on; the left-to-right sweep then
  // contracts W_k with Q_k by a GEMM instead of applying the tree
  void* Qx[TT_MAXD] = {nullptr};
  double* eye = nullptr;
  int64_t eye_n = 0;            // the identity is eye_n x eye_n (the widest core with an explicit Q)
  char* qx_block = nullptr;
  size_t qx_cap = 0;
  // planning at rank bounds: the result's cores at their bound shapes (core k at stg_off[k])
  char* stage = nullptr;
  int64_t stg_off[TT_MAXD] = {0};
};

#ifndef TT_QX_MAX_COLS
#define TT_QX_MAX_COLS 256
#endif
constexpr int64_t QX_MAX_COLS = TT_QX_MAX_COLS;   // explicit orthogonal factors of at most this many columns

// Bytes a tree plan of any M' x N matrix with M' <= M needs, whatever shape the
// autotuner picks for it: the most storage goes to the shape with the
// shortest leaves (N rows) and fan-in 2 (most stacked triangles), so that
// shape is measured.  (Used where the row count is known only as a bound.)
TreeShape worst_shape(int64_t M, int64_t N) {
  TreeShape sh;
  sh.leaf_rows = (int32_t)std::min<int64_t>(std::max<int64_t>(N, 1), QR_MAXROWS);
  sh.fanin = 2;
  if (M <= QR_MAXROWS && N >= M) sh.leaf_rows = (int32_t)M;
  return sh;
}

size_t tree_bytes(int64_t M, int64_t N, int dtype) {
  size_t best = 0;
  for (int pass = 0; pass < 2; ++pass) {   // the default/tuned plan and the worst legal shape
    Carver cv;
    cv.measure = true;
    Tree t;
    const bool ok = pass == 0 ? plan_tree(cv, t, M, N, dtype, nullptr, 1, 1, nullptr)
                              : plan_tree_shape(cv, t, M, N, dtype, nullptr, 1, 1, worst_shape(M, N), nullptr);
    if (!ok) return 0;
    best = std::max(best, cv.off);
  }
  return best;
}

size_t tree_apply_bytes(int64_t M, int64_t N, int dtype, int64_t tcols) {
  size_t best = 0;
  for (int pass = 0; pass < 2; ++pass) {
    Carver cv;
    cv.measure = true;
    Tree t;
    const bool ok = pass == 0 ? plan_tree(cv, t, M, N, dtype, nullptr, 1, 1, nullptr)
                              : plan_tree_shape(cv, t, M, N, dtype, nullptr, 1, 1, worst_shape(M, N), nullptr);
    if (!ok) return 0;
    best = std::max(best, apply_work_bytes(t, tcols));
  }
  return best;
}

// plan buffers of one job (workspace carving); returns false on unsupported shape
bool plan_job(tt_ctx* c, RJob& jb, JobState& st, std::string* why, bool bound_plan = false) {
  const int d = jb.d;
  const size_t elt = elt_size(jb.dtype);
  st.s[d] = 1;
  for (int k = d - 1; k >= 1; --k) st.s[k] = std::min<int64_t>(jb.R[k], jb.n[k] * st.s[k + 1]);
  st.s[0] = 1;
  st.tb[0] = 1;
  for (int k = 0; k + 1 < d; ++k) {
    int64_t b = std::min<int64_t>(st.tb[k] * jb.n[k], st.s[k + 1]);
    if (jb.max_rank > 0) b = std::min<int64_t>(b, jb.max_rank);
    st.tb[k + 1] = std::max<int64_t>(b, 1);
  }
  st.tb[d] = 1;
  Carver ws;
  ws.ctx = c;
  for (int k = d - 1; k >= 1; --k) {
    const int64_t M = jb.n[k] * st.s[k + 1], N = jb.R[k];
    st.Y[k] = ws.take((size_t)M * N * elt);
    if (!plan_tree(ws, st.rl[k], M, N, jb.dtype, st.Y[k], 1, M, why)) return false;
  }
  // C buffer, L-to-R tree block, SVD buffers, apply scratch
  size_t cmax = 0, lrmax = 0, apmax = 0;
  int64_t smax = 1, tmax = 1;
  for (int k = 0; k + 1 < d; ++k) {
    const int64_t M = st.tb[k] * jb.n[k], N = st.s[k + 1];
    cmax = std::max(cmax, (size_t)(M * N));
    const size_t tb = tree_bytes(M, N, jb.dtype);
    if (tb == 0) {
      Carver tmp;
      tmp.measure = true;
      Tree tt;
      plan_tree(tmp, tt, M, N, jb.dtype, nullptr, 1, 1, why);
      return false;
    }
    lrmax = std::max(lrmax, tb);
    apmax = std::max(apmax, tree_apply_bytes(M, N, jb.dtype, st.tb[k + 1]));
    smax = std::max(smax, N);
    tmax = std::max(tmax, st.tb[k + 1]);
    // the SVD takes R factors of at most SVD_BIG_MAX rows (one workgroup up to
    // SVD_SMALL_MAX); planned at the rank bounds every step stays within the one-workgroup
    // kernel; planned at the chosen ranks, each step is checked when its rank is known
    if (bound_plan && std::min(M, N) > SVD_SMALL_MAX) {
      if (why)
        *why = "SVD of a " + std::to_string(std::min(M, N)) + "-row R factor exceeds " + std::to_string(SVD_SMALL_MAX);
      return false;
    }
  }
  for (int k = 1; k < d; ++k) apmax = std::max(apmax, apply_work_bytes(st.rl[k], st.tb[k]));
  st.C = ws.take(std::max<size_t>(cmax, 1) * elt);
  st.lr_cap = lrmax;
  st.lr_blk[0] = (char*)ws.take(std::max<size_t>(lrmax, 256));
  st.lr_blk[1] = (char*)ws.take(std::max<size_t>(lrmax, 256));
  st.ap_cap = apmax;
  st.ap_block = (char*)ws.take(std::max<size_t>(apmax, 256));
  st.ap_side = (char*)ws.take(std::max<size_t>(apmax, 256));
  st.A = (double*)ws.take((size_t)smax * smax * 8);
  st.acc = (double*)ws.take((size_t)smax * smax * 8);
  st.sig = (double*)ws.take((size_t)smax * 8);
  st.perm = (int32_t*)ws.take((size_t)smax * 4);
  st.iscr = (int32_t*)ws.take((size_t)(2 * smax + 128) * 4);
  st.wt = (double*)ws.take((size_t)smax * tmax * 8);
  st.urb[0] = (double*)ws.take((size_t)smax * tmax * 8);
  st.urb[1] = (double*)ws.take((size_t)smax * tmax * 8);
  st.d_norm = (double*)ws.take(64);
  // explicit Q for the right-to-left cores 2..d-1 (core 1's is needed right after the sweep,
  // so it keeps the tree application); one identity and one apply scratch shared by them.
  // Only for factors of at most QX_MAX_COLS columns: forming Q applies the tree to s_k
  // columns, the left-to-right step then needs t_k <= s_k of them, so for wide factors of
  // low truncated rank the direct application is far cheaper (and needs no M x s_k copy).
  int64_t nmax = 0;
  size_t qx_work = 0;
  for (int k = 2; k < d; ++k) {
    const int64_t M = jb.n[k] * st.s[k + 1], N = jb.R[k];
    if (st.s[k] > QX_MAX_COLS) continue;
    st.Qx[k] = ws.take((size_t)M * st.s[k] * elt);
    nmax = std::max(nmax, N);
    qx_work = std::max(qx_work, apply_work_bytes(st.rl[k], N));
  }
  if (nmax > 0) {
    st.eye = (double*)ws.take((size_t)nmax * nmax * 8);
    st.eye_n = nmax;
    st.qx_cap = qx_work;
    st.qx_block = (char*)ws.take(std::max<size_t>(qx_work, 256));
  }
  if (bound_plan) {
    // cores at their bound shapes: in the output itself when it holds them (then only cores
    // whose ranks fall below the bounds move), else in a workspace staging area
    int64_t tot = 0;
    for (int k = 0; k < d; ++k) {
      st.stg_off[k] = tot;
      tot += st.tb[k] * jb.n[k] * st.tb[k + 1];
    }
    if (jb.out && jb.out->capacity >= tot) st.stage = (char*)jb.out->data;
    else st.stage = (char*)ws.take((size_t)std::max<int64_t>(tot, 1) * elt);
  }
  return true;
}

tt_status launch_levels_plain(tt_ctx* c, std::vector<Tree*>& trees) {
  // level by level from the leaves, all trees together (grouped by dtype)
  int maxL = 0;
  for (Tree* t : trees) maxL = std::max(maxL, t->depth());
  for (int l = 0; l < maxL; ++l) {
    for (int pass = 0; pass < 2; ++pass) {   // pass 0: FP64 tiles, pass 1: FP32 tiles
      // group by (child dtype) for nodes: children of level-1 nodes are leaves
      for (int srcd = 0; srcd < 2; ++srcd) {
        std::vector<QrTask> tasks;
        std::vector<QrTask> children;
        for (Tree* t : trees) {
          if (l >= t->depth()) continue;
          const int tile_d = (l == 0) ? t->leaf_dtype : TT_F64;
          const int src_d = (l == 0) ? t->leaf_dtype : (l == 1 ? t->leaf_dtype : TT_F64);
          if ((tile_d == TT_F64) != (pass == 0) || src_d != srcd) continue;
          const int base = (int)children.size();
          if (l > 0) children.insert(children.end(), t->lvl[l - 1].begin(), t->lvl[l - 1].end());
          for (QrTask q : t->lvl[l]) {
            if (l > 0) q.child0 += base;
            tasks.push_back(q);
          }
        }
        if (tasks.empty()) continue;
        const QrTask *dt = nullptr, *dc = nullptr;
        if (!upload_pair(c, tasks, children, &dt, &dc) || !dt) return fail(c, TT_ENOMEM, "task upload");
        double fl = 0.0, by = 0.0;
        if (c->prof)
          for (const QrTask& q : tasks) {
            fl += qr_flops(q);
            by += 2.0 * (double)q.m * q.ncol * (pass == 0 ? 8.0 : 4.0);
          }
        const int pr = prof_begin(c, l == 0 ? PK_QR_LEAF : PK_QR_NODE, fl, by);
        int max_rows = 1;
        for (const QrTask& q : tasks) max_rows = std::max(max_rows, (int)q.m);
        hipError_t e = launch_qr_factor(srcd, pass == 0 ? 0 : 1, dt, dc, (int)tasks.size(), max_rows, c->stream);
        prof_end(c, pr);
        if (e != hipSuccess) return hip_fail(c, e, "qr_factor");
      }
    }
    // column blocks: the carried columns of this level's tiles updated by their reflectors,
    // one workgroup per 16 columns of a tile, before the next level stacks them
    for (int tdt = 0; tdt < 2; ++tdt) {
      std::vector<ApplyTask> up;
      int max_rows = 1, max_t = 0;
      for (Tree* t : trees) {
        if (l >= t->depth() || !t->next) continue;
        const int tile_d = (l == 0) ? t->leaf_dtype : TT_F64;
        if (tile_d != tdt) continue;
        for (const QrTask& q : t->lvl[l]) {
          ApplyTask a;
          std::memset(&a, 0, sizeof(a));
          a.tile = q.tile;
          a.tau = q.tau;
          a.tmat = q.tmat;
          a.m = q.m;
          a.ncol = q.ncol;
          a.kq = (int32_t)std::min<int64_t>(q.m, q.nfact);
          a.nchild = q.nchild;
          a.kc0 = q.kc0;
          a.kc_last = q.kc_last;
          a.t = q.ncol - q.nfact;
          a.out = (char*)q.tile + (size_t)q.nfact * elt_size(tile_d);
          a.out_rs = q.ncol;
          a.out_cs = 1;
          up.push_back(a);
          max_rows = std::max(max_rows, (int)q.m);
          max_t = std::max(max_t, (int)a.t);
        }
      }
      if (up.empty()) continue;
      const ApplyTask* du = upload(c, up);
      if (!du) return fail(c, TT_ENOMEM, "task upload");
      double fl = 0.0;
      if (c->prof)
        for (const ApplyTask& a : up) fl += apply_flops(a);
      const int pr = prof_begin(c, PK_QR_APPLY, fl, 0.0);
      const hipError_t e = launch_qr_update(tdt, du, (int)up.size(), max_rows, max_t, c->stream);
      prof_end(c, pr);
      if (e != hipSuccess) return hip_fail(c, e, "qr_update");
    }
  }
  return TT_OK;
}

tt_status launch_copies(tt_ctx* c, const std::vector<BlockCopy>& cp) {
  if (cp.empty()) return TT_OK;
  const BlockCopy* d = upload(c, cp);
  if (!d) return fail(c, TT_ENOMEM, "task upload");
  int64_t rows = 1;
  for (const BlockCopy& b : cp) rows = std::max<int64_t>(rows, b.rows);
  const int pr = prof_begin(c, PK_OTHER, 0.0, 0.0);
  const hipError_t e = launch_block_copy(d, (int)cp.size(), rows, c->stream);
  prof_end(c, pr);
  return e == hipSuccess ? TT_OK : hip_fail(c, e, "block copy");
}

// Factorisation of trees, column-blocked ones included: the tiles of every tree level by
// level; for blocked trees then the left-behind rows gathered, the block's rows of R copied
// out and each tile's factored columns moved to its compact tile (the shared full-width
// region is free after that), the trailing blocks factored the same way, and the trailing
// R copied in where the trailing block is an ordinary tree (a blocked one wrote it in place).
tt_status launch_levels_factor(tt_ctx* c, std::vector<Tree*>& trees) {
  tt_status st = launch_levels_plain(c, trees);
  if (st != TT_OK) return st;
  std::vector<Tree*> blocked, nexts;
  for (Tree* t : trees)
    if (t->next) {
      blocked.push_back(t);
      nexts.push_back(t->next.get());
    }
  if (blocked.empty()) return TT_OK;
  std::vector<BlockCopy> cp;
  for (Tree* t : blocked) {
    const std::vector<std::vector<int64_t>> off = rest_offsets(*t);
    const int64_t nf = t->nf, N = t->N, wc = N - nf, ld = t->r_ld;
    for (size_t l = 0; l < t->lvl.size(); ++l) {
      const int tdt = l == 0 ? t->leaf_dtype : TT_F64;
      for (size_t i = 0; i < t->lvl[l].size(); ++i) {
        const QrTask& q = t->lvl[l][i];
        const int64_t k = std::min<int64_t>(q.m, nf);
        BlockCopy b;
        std::memset(&b, 0, sizeof(b));
        b.src = q.tile;   // the factored columns, kept for the application of Q
        b.src_ld = N;
        b.dst = t->ctile[l][i];
        b.dst_ld = nf;
        b.rows = q.m;
        b.cols = (int32_t)nf;
        b.src_f32 = b.dst_f32 = tdt == TT_F32;
        cp.push_back(b);
        if (q.m <= k) continue;
        std::memset(&b, 0, sizeof(b));   // the left-behind rows of the carried columns
        b.src = (const char*)q.tile + (size_t)(k * N + nf) * elt_size(tdt);
        b.src_ld = N;
        b.dst = (char*)t->rest + (size_t)(off[l][i] * wc) * elt_size(t->leaf_dtype);
        b.dst_ld = wc;
        b.rows = (int32_t)(q.m - k);
        b.cols = (int32_t)wc;
        b.src_f32 = tdt == TT_F32;
        b.dst_f32 = t->leaf_dtype == TT_F32;
        cp.push_back(b);
      }
    }
    const QrTask& root = t->lvl.back()[0];
    const int64_t k2 = std::min(t->M, N) - nf;
    BlockCopy b;
    std::memset(&b, 0, sizeof(b));
    b.src = root.tile;   // rows 0..nf-1: [R_11 R_12]
    b.src_ld = N;
    b.src_f32 = t->lvl.size() == 1 && t->leaf_dtype == TT_F32;
    b.dst = t->rfull;
    b.dst_ld = ld;
    b.rows = (int32_t)nf;
    b.cols = (int32_t)N;
    b.tri = 1;
    cp.push_back(b);
    std::memset(&b, 0, sizeof(b));   // rows nf..kr-1, columns 0..nf-1: zero
    b.dst = t->rfull + nf * ld;
    b.dst_ld = ld;
    b.rows = (int32_t)k2;
    b.cols = (int32_t)nf;
    cp.push_back(b);
  }
  if ((st = launch_copies(c, cp)) != TT_OK) return st;
  if ((st = launch_levels_factor(c, nexts)) != TT_OK) return st;
  cp.clear();
  for (Tree* t : blocked) {
    if (t->next->next) continue;   // a blocked trailing block wrote its R in place
    const int64_t nf = t->nf, N = t->N, ld = t->r_ld, k2 = t->next->kr();
    BlockCopy b;
    std::memset(&b, 0, sizeof(b));   // rows nf..kr-1, columns nf..N-1: R of the trailing block
    b.src = t->next->root_R();
    b.src_ld = t->next->rld();
    b.src_f32 = t->next->root_f32();
    b.dst = t->rfull + nf * ld + nf;
    b.dst_ld = ld;
    b.rows = (int32_t)k2;
    b.cols = (int32_t)(N - nf);
    b.tri = 1;
    cp.push_back(b);
  }
  return launch_copies(c, cp);
}

tt_status launch_apply_plans(tt_ctx* c, std::vector<std::vector<ApplyLevel>>& plans, int out_dtype,
                             hipStream_t stream = nullptr) {
  if (!stream) stream = c->stream;
  int maxL = 0;
  for (auto& p : plans) maxL = std::max(maxL, (int)p.size());
  for (int depth = 0; depth < maxL; ++depth) {
    for (int tdt = 0; tdt < 2; ++tdt) {
      std::vector<ApplyTask> tasks;
      for (auto& p : plans) {
        if (depth >= (int)p.size()) continue;
        if (p[depth].tile_dtype != tdt) continue;
        tasks.insert(tasks.end(), p[depth].tasks.begin(), p[depth].tasks.end());
      }
      if (tasks.empty()) continue;
      const ApplyTask* dt = upload(c, tasks);
      if (!dt) return fail(c, TT_ENOMEM, "task upload");
      double fl = 0.0, by = 0.0;
      if (c->prof)
        for (const ApplyTask& a : tasks) {
          fl += apply_flops(a);
          by += (double)a.m * a.ncol * (tdt == 0 ? 8.0 : 4.0) + 2.0 * (double)a.m * a.t * 8.0;
        }
      const int pr = prof_begin(c, PK_QR_APPLY, fl, by, stream);
      int max_rows = 1, max_t = 0;
      for (const ApplyTask& a : tasks) {
        max_rows = std::max(max_rows, (int)a.m);
        max_t = std::max(max_t, (int)a.t);
      }
      hipError_t e = launch_qr_apply(tdt, out_dtype, dt, (int)tasks.size(), max_rows, max_t, stream);
      prof_end(c, pr, stream);
      if (e != hipSuccess) return hip_fail(c, e, "qr_apply");
    }
  }
  return TT_OK;
}

}  // namespace

tt_status tune_tree(tt_ctx* c, int64_t M, int64_t N, int dtype, TreeShape* best_out) {
  const TreeShape def = default_shape(M, N);
  if (best_out) *best_out = def;
  if (M < 1 || N < 1) return TT_OK;
  // candidate leaf heights: the whole matrix when it fits one tile, and multiples of N
  std::vector<int64_t> bs;
  if (M <= QR_MAXROWS) bs.push_back(M);
  for (double f : {1.0, 1.5, 2.0, 3.0, 4.0, 6.0}) {
    int64_t b = ((int64_t)std::ceil(f * (double)std::max<int64_t>(N, 16)) + 15) / 16 * 16;
    if (b >= N && b <= QR_MAXROWS && b < M) bs.push_back(b);
  }
  for (int64_t b : {256, 512, 768})
    if (b >= N && b < M) bs.push_back(b);
  std::sort(bs.begin(), bs.end());
  bs.erase(std::unique(bs.begin(), bs.end()), bs.end());
  std::vector<TreeShape> cand;
  for (int64_t b : bs) {
    const int64_t kc = std::min<int64_t>(b, N);
    if (b >= M) {
      cand.push_back(TreeShape{(int32_t)b, def.fanin});
      continue;
    }
    for (int64_t g : {2, 3, 4, 6, 8, 12, 16})
      if (g * kc <= QR_MAXROWS) cand.push_back(TreeShape{(int32_t)b, (int32_t)g});
  }
  if (cand.empty()) return TT_OK;
  ++c->tune_count;
  const size_t elt = elt_size(dtype);
  const size_t mark = c->ws_off;
  struct Reset {
    tt_ctx* c;
    size_t off;
    ~Reset() { c->ws_off = off; }
  } reset{c, mark};
  const bool overflow0 = c->ws_overflow;
  void* src = ws_alloc(c, (size_t)M * N * elt);
  if (!src) {
    c->ws_overflow = overflow0;
    return TT_OK;   // no room to tune here: the default shape stays in use
  }
  hipError_t e = launch_fill_pattern(dtype, src, M * N, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "tune fill");
  hipEvent_t e0, e1;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(c, e, "tune event");
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(c, e, "tune event");
  }
  const bool prof = c->prof;
  c->prof = false;
  TreeShape best = def;
  float best_ms = 1e30f, def_ms = 1e30f;
  tt_status st = TT_OK;
  for (const TreeShape& sh : cand) {
    const size_t m2 = c->ws_off;
    Carver cv;
    cv.ctx = c;
    Tree t;
    if (!plan_tree_shape(cv, t, M, N, dtype, src, 1, M, sh, nullptr) || c->ws_overflow) {
      c->ws_overflow = overflow0;
      c->ws_off = m2;
      continue;
    }
    std::vector<Tree*> tv(1, &t);
    // the tree is timed as TT-round uses it: factorisation, then the application of
    // its Q to a block of min(N, 32) columns (the left-to-right sweep)
    const int64_t tcols = std::min<int64_t>(N, 32);
    Carver acv;
    acv.ctx = c;
    std::vector<std::vector<ApplyLevel>> plans(1);
    double* X = (double*)ws_alloc(c, (size_t)N * tcols * 8);
    void* out = ws_alloc(c, (size_t)M * tcols * elt);
    if (!X || !out || c->ws_overflow) {
      c->ws_overflow = overflow0;
      c->ws_off = m2;
      continue;
    }
    plan_apply(acv, t, X, tcols, tcols, out, dtype, tcols, 1, plans[0]);
    if (c->ws_overflow) {
      c->ws_overflow = overflow0;
      c->ws_off = m2;
      continue;
    }
    if ((e = launch_fill_pattern(TT_F64, X, N * tcols, c->stream)) != hipSuccess) { st = hip_fail(c, e, "tune"); break; }
    float ms = 1e30f;
    for (int rep = 0; rep < 5 && st == TT_OK; ++rep) {
      if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) { st = hip_fail(c, e, "tune"); break; }
      if ((st = launch_levels_factor(c, tv)) != TT_OK) break;
      if ((st = launch_apply_plans(c, plans, dtype)) != TT_OK) break;
      if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) { st = hip_fail(c, e, "tune"); break; }
      if ((e = hipEventSynchronize(e1)) != hipSuccess) { st = hip_fail(c, e, "tune"); break; }
      float x = 0.f;
      if (rep > 0 && hipEventElapsedTime(&x, e0, e1) == hipSuccess) ms = std::min(ms, x);
    }
    c->ws_off = m2;
    if (st != TT_OK) break;
    const bool is_def = sh.leaf_rows == def.leaf_rows && (sh.fanin == def.fanin || sh.leaf_rows >= M);
    if (is_def) def_ms = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = sh;
    }
  }
  // keep the default shape unless another one is clearly (5%) faster: timing noise
  // must not move the choice
  if (def_ms < 1e29f && best_ms > 0.95f * def_ms) best = def;
  c->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != TT_OK) return st;
  set_tuned_shape(M, N, dtype, best);
  if (best_out) *best_out = best;
  return TT_OK;
}

tt_status round_jobs_grouped(tt_ctx* c, std::vector<RJob>& jobs) {
  if (jobs.size() <= 1) return round_jobs(c, jobs);
  std::vector<int64_t> need(jobs.size());
  int64_t big = 0;
  for (size_t i = 0; i < jobs.size(); ++i) {
    std::vector<RJob> one(1, jobs[i]);
    need[i] = std::max<int64_t>(round_workspace_bytes(one), 0);
    big = std::max(big, need[i]);
  }
  const int64_t lim = std::max<int64_t>(big, (int64_t)32 << 30);
  if (c->ws_off + (size_t)big > c->ws_bytes) {   // report the largest group's need at once
    c->required = std::max(c->required, c->ws_off + (size_t)std::min<int64_t>(lim, [&] {
      int64_t t = 0;
      for (int64_t v : need) t += v;
      return t;
    }()));
    return fail(c, TT_ECAPACITY, "workspace too small for the batched roundings: need " + std::to_string(c->required));
  }
  size_t i0 = 0;
  while (i0 < jobs.size()) {
    size_t i1 = i0;
    int64_t sum = 0;
    while (i1 < jobs.size() && (i1 == i0 || sum + need[i1] <= lim)) sum += need[i1++];
    std::vector<RJob> grp(jobs.begin() + i0, jobs.begin() + i1);
    const tt_status s = round_jobs(c, grp);
    if (s != TT_OK) return s;
    for (size_t k = i0; k < i1; ++k) {   // what round_jobs reports back in a job
      jobs[k].status = grp[k - i0].status;
      jobs[k].norm = grp[k - i0].norm;
    }
    i0 = i1;
  }
  return TT_OK;
}

int64_t round_workspace_bytes(const std::vector<RJob>& jobs) {
  tt_ctx tmp;
  tmp.ws = nullptr;
  tmp.ws_bytes = 0;
  tmp.ws_off = 0;
  std::vector<JobState> st(jobs.size());
  for (size_t j = 0; j < jobs.size(); ++j) {
    RJob jb = jobs[j];
    if (jb.d >= 2) {
      std::string why;
      if (!plan_job(&tmp, jb, st[j], &why)) return -1;
    }
  }
  return (int64_t)tmp.ws_off + 4096;
}

tt_status round_jobs(tt_ctx* c, std::vector<RJob>& jobs, const RoundMode& mode) {
  if (jobs.empty()) return TT_OK;
  const bool bp = mode.bound_plan;
  const int dtype = jobs[0].dtype;
  for (const RJob& jb : jobs)
    if (jb.dtype != dtype) return fail(c, TT_EINVAL, "all jobs of a batch must share one dtype");
  const size_t elt = elt_size(dtype);
  hipStream_t s = c->stream;
  hipError_t e;
  const int nj = (int)jobs.size();
  std::vector<JobState> st(nj);

  // ---------------- plan all buffers before any launch (workspace released on return)
  struct WsMark {
    tt_ctx* c;
    size_t off;
    ~WsMark() { c->ws_off = off; }
  } mark{c, c->ws_off};
  c->ws_overflow = false;
  if (c->autotune) {
    // shapes of the right-to-left trees (the left-to-right ones are tuned when their rank is known)
    for (int j = 0; j < nj; ++j) {
      const RJob& jb = jobs[j];
      if (jb.d < 2) continue;
      int64_t s1 = 1;
      for (int k = jb.d - 1; k >= 1; --k) {
        const int64_t M = jb.n[k] * s1, N = jb.R[k];
        if (!tuned_shape(M, N, jb.dtype, nullptr)) {
          tt_status ts = tune_tree(c, M, N, jb.dtype, nullptr);
          if (ts != TT_OK) return ts;
        }
        s1 = std::min<int64_t>(jb.R[k], jb.n[k] * s1);
      }
    }
  }
  for (int j = 0; j < nj; ++j) {
    RJob& jb = jobs[j];
    int64_t need = 0;
    if (jb.d == 1) {
      need = jb.n[0];
      if (jb.orth_only) st[j].C = ws_alloc(c, (size_t)jb.n[0] * elt);   // the materialised sum
    } else {
      std::string why;
      if (!plan_job(c, jb, st[j], &why, bp && !jb.orth_only)) return fail(c, TT_ENOTIMPL, why);
      int64_t b = 0;
      for (int k = 0; k < jb.d; ++k) b += st[j].tb[k] * jb.n[k] * st[j].tb[k + 1];
      need = b;
    }
    (void)need;
  }
  if (bp && c->autotune) {
    // planning at the bounds knows every left-to-right shape now: tune them before any launch
    for (int j = 0; j < nj; ++j) {
      const RJob& jb = jobs[j];
      for (int k = 0; k + 1 < jb.d; ++k) {
        const int64_t M = st[j].tb[k] * jb.n[k], N = st[j].s[k + 1];
        if (!tuned_shape(M, N, jb.dtype, nullptr)) {
          tt_status ts = tune_tree(c, M, N, jb.dtype, nullptr);
          if (ts != TT_OK) return ts;
        }
      }
    }
  }
  if (c->ws_overflow) {
    c->required = std::max(c->required, c->ws_off);
    return fail(c, TT_ECAPACITY, "workspace too small: need " + std::to_string(c->ws_off) + " bytes, have " +
                                     std::to_string(c->ws_bytes));
  }
  int32_t* d_ranks = (int32_t*)dev_scratch(c, (size_t)nj * (TT_MAXD + 1) * 4);
  int32_t* h_ranks = (int32_t*)c->pin.alloc((size_t)nj * (TT_MAXD + 1) * 4);
  double* h_norms = (double*)c->pin.alloc((size_t)nj * 8);
  double* d_norms = (double*)dev_scratch(c, (size_t)nj * 8);   // ||x|| of every job, read back at once
  if (!d_ranks || !h_ranks || !h_norms || !d_norms) return fail(c, TT_ENOMEM, "small buffers");
  for (int j = 0; j < nj; ++j) st[j].d_norm = d_norms + j;

  // ---------------- order-1 jobs: the sum itself (components accumulated in order)
  {
    size_t maxc = 0;
    for (int j = 0; j < nj; ++j) {
      RJob& jb = jobs[j];
      if (jb.d != 1) continue;
      if (!jb.orth_only && jb.out->capacity < jb.n[0]) jb.status = TT_ECAPACITY;
      else maxc = std::max(maxc, jb.comps.size());
    }
    for (size_t ci = 0; ci < maxc; ++ci) {
      std::vector<CopySeg> g;
      for (int j = 0; j < nj; ++j) {
        RJob& jb = jobs[j];
        if (jb.d != 1 || jb.status != TT_OK || ci >= jb.comps.size()) continue;
        CopySeg sg;
        sg.src = jb.comps[ci].data;
        sg.dst = jb.orth_only ? st[j].C : jb.out->data;
        sg.count = jb.n[0];
        sg.coef = jb.comps[ci].coef;
        sg.accumulate = ci > 0;
        g.push_back(sg);
      }
      if (g.empty()) continue;
      const CopySeg* dg = upload(c, g);
      if (!dg) return fail(c, TT_ENOMEM, "task upload");
      if ((e = launch_copy_segs(dtype, dg, (int)g.size(), s)) != hipSuccess) return hip_fail(c, e, "copy");
    }
    std::vector<SumsqTask> nt;
    for (int j = 0; j < nj; ++j) {
      RJob& jb = jobs[j];
      if (jb.d != 1 || jb.status != TT_OK) continue;
      nt.push_back(SumsqTask{jb.orth_only ? st[j].C : jb.out->data, jb.n[0], st[j].d_norm});
    }
    if (!nt.empty()) {
      const SumsqTask* dn = upload(c, nt);
      if (!dn) return fail(c, TT_ENOMEM, "task upload");
      if ((e = launch_sumsq_batched(dtype, dn, (int)nt.size(), s)) != hipSuccess) return hip_fail(c, e, "sumsq");
    }
  }

  // ---------------- right-to-left sweep
  {
    std::vector<CopySeg> segs;
    for (int j = 0; j < nj; ++j) {
      RJob& jb = jobs[j];
      if (jb.d < 2) continue;
      const int k = jb.d - 1;
      for (size_t ci = 0; ci < jb.comps.size(); ++ci) {
        const Comp& cp = jb.comps[ci];
        CopySeg sg;
        sg.src = cp.data + (size_t)cp.core_off[k] * elt;
        sg.dst = (char*)st[j].Y[k] + (size_t)(jb.roff[ci * (jb.d + 1) + k] * jb.n[k]) * elt;
        sg.count = cp.r[k] * jb.n[k];
        sg.coef = 1.0;
        sg.accumulate = 0;
        segs.push_back(sg);
      }
    }
    if (!segs.empty()) {
      const CopySeg* dg = upload(c, segs);
      if (!dg) return fail(c, TT_ENOMEM, "task upload");
      if ((e = launch_copy_segs(dtype, dg, (int)segs.size(), s)) != hipSuccess) return hip_fail(c, e, "gather");
    }
  }
  int maxd = 0;
  for (const RJob& jb : jobs) maxd = std::max(maxd, jb.d);
  std::vector<hipEvent_t> qx_done(maxd, nullptr);   // side-stream completion of the explicit Q of a step
  // one identity for every job's explicit Q: the largest of the jobs' identity buffers
  double* eye = nullptr;
  int64_t eye_n = 0;
  for (int j = 0; j < nj; ++j)
    if (st[j].eye && st[j].eye_n > eye_n) {   // (sized in plan_job: only cores with an explicit Q)
      eye_n = st[j].eye_n;
      eye = st[j].eye;
    }
  if (eye && (e = launch_eye(eye, (int)eye_n, s)) != hipSuccess) return hip_fail(c, e, "eye");
  for (int step = 0; step + 1 < maxd; ++step) {
    std::vector<Tree*> trees;
    std::vector<int> act;
    for (int j = 0; j < nj; ++j) {
      const int k = jobs[j].d - 1 - step;
      if (jobs[j].d >= 2 && k >= 1) {
        trees.push_back(&st[j].rl[k]);
        act.push_back(j);
      }
    }
    if (act.empty()) continue;
    tt_status rs = launch_levels_factor(c, trees);
    if (rs != TT_OK) return rs;
    // explicit Q_k of cores 2..d-1 on the side stream: the tree applied to the identity
    {
      std::vector<std::vector<ApplyLevel>> xplans;
      for (int j : act) {
        const int k = jobs[j].d - 1 - step;
        JobState& js = st[j];
        if (k < 2 || !js.Qx[k]) continue;
        const int64_t sk = js.s[k];   // columns of Q_k: min(R_k, n_k s_{k+1})
        Carver cv;
        cv.base = js.qx_block;
        cv.cap = js.qx_cap;
        std::vector<ApplyLevel> pl;
        plan_apply(cv, js.rl[k], eye, eye_n, sk, js.Qx[k], jobs[j].dtype, sk, 1, pl);
        if (cv.off > cv.cap) return fail(c, TT_ECAPACITY, "explicit Q scratch");
        xplans.push_back(std::move(pl));
      }
      if (!xplans.empty()) {
        hipStream_t side = side_stream(c);
        hipEvent_t ready = dep_event(c), done = dep_event(c);
        if (!side || !ready || !done) return fail(c, TT_EDEVICE, "side stream");
        if ((e = hipEventRecord(ready, s)) != hipSuccess) return hip_fail(c, e, "event");
        if ((e = hipStreamWaitEvent(side, ready, 0)) != hipSuccess) return hip_fail(c, e, "event");
        c->upload_stream = side;
        rs = launch_apply_plans(c, xplans, dtype, side);
        c->upload_stream = nullptr;
        if (rs != TT_OK) return rs;
        if ((e = hipEventRecord(done, side)) != hipSuccess) return hip_fail(c, e, "event");
        qx_done[step] = done;
      }
    }
    // contraction into core k-1
    std::vector<GemmTask> gt;
    std::vector<GemmPart> gp;
    int max_m = 0, max_n = 0;
    for (int j : act) {
      RJob& jb = jobs[j];
      JobState& js = st[j];
      const int k = jb.d - 1 - step;
      const Tree& tr = js.rl[k];
      const int D = jb.d + 1;
      if (k - 1 >= 1) {
        for (size_t ci = 0; ci < jb.comps.size(); ++ci) {
          const Comp& cp = jb.comps[ci];
          GemmTask g;
          std::memset(&g, 0, sizeof(g));
          g.M = (int32_t)(cp.r[k - 1] * jb.n[k - 1]);
          g.N = (int32_t)js.s[k];
          g.part0 = (int32_t)gp.size();
          g.nparts = 1;
          g.B = tr.root_R();
          g.b_ld = tr.rld();
          g.b_f32 = tr.root_f32();
          g.C = (char*)js.Y[k - 1] + (size_t)(jb.roff[ci * D + (k - 1)] * jb.n[k - 1] * js.s[k]) * elt;
          g.c_ld = js.s[k];
          GemmPart p;
          p.A = cp.data + (size_t)cp.core_off[k - 1] * elt;
          p.K = (int32_t)cp.r[k];
          p.b_off = (int32_t)jb.roff[ci * D + k];
          p.coef = 1.0;
          gp.push_back(p);
          gt.push_back(g);
          max_m = std::max(max_m, g.M);
          max_n = std::max(max_n, g.N);
        }
      } else {
        GemmTask g;
        std::memset(&g, 0, sizeof(g));
        g.M = (int32_t)jb.n[0];
        g.N = (int32_t)js.s[1];
        g.part0 = (int32_t)gp.size();
        g.nparts = (int32_t)jb.comps.size();
        g.B = tr.root_R();
        g.b_ld = tr.rld();
        g.b_f32 = tr.root_f32();
        g.C = js.C;
        g.c_ld = js.s[1];
        for (size_t ci = 0; ci < jb.comps.size(); ++ci) {
          const Comp& cp = jb.comps[ci];
          GemmPart p;
          p.A = cp.data + (size_t)cp.core_off[0] * elt;
          p.K = (int32_t)cp.r[1];
          p.b_off = (int32_t)jb.roff[ci * D + 1];
          p.coef = cp.coef;
          gp.push_back(p);
        }
        gt.push_back(g);
        max_m = std::max(max_m, g.M);
        max_n = std::max(max_n, g.N);
      }
    }
    const GemmTask* dgt = nullptr;
    const GemmPart* dgp = nullptr;
    if (!upload_pair(c, gt, gp, &dgt, &dgp)) return fail(c, TT_ENOMEM, "task upload");
    double gfl = 0.0, gby = 0.0;
    for (const GemmTask& g : gt)
      for (int pi = 0; pi < g.nparts; ++pi) {
        gfl += 2.0 * g.M * g.N * (double)gp[g.part0 + pi].K;
        gby += (double)elt * ((double)g.M * gp[g.part0 + pi].K) + 8.0 * g.N * (double)gp[g.part0 + pi].K;
      }
    for (const GemmTask& g : gt) gby += (double)elt * g.M * g.N;
    const int gpr = prof_begin(c, PK_GEMM, gfl, gby);
    e = launch_gemm(dtype, dgt, dgp, (int)gt.size(), max_m, max_n, s);
    prof_end(c, gpr);
    if (e != hipSuccess) return hip_fail(c, e, "contraction");
  }

  // ---------------- norms
  {
    std::vector<SumsqTask> nt;
    for (int j = 0; j < nj; ++j) {
      RJob& jb = jobs[j];
      if (jb.d < 2) continue;
      nt.push_back(SumsqTask{st[j].C, jb.n[0] * st[j].s[1], st[j].d_norm});
    }
    if (!nt.empty()) {
      const SumsqTask* dn = upload(c, nt);
      if (!dn) return fail(c, TT_ENOMEM, "task upload");
      if ((e = launch_sumsq_batched(dtype, dn, (int)nt.size(), s)) != hipSuccess) return hip_fail(c, e, "norm");
    }
  }

  // ---------------- left-to-right sweep
  for (int j = 0; j < nj; ++j) {
    st[j].t[0] = 1;
    st[j].out_off = 0;
    st[j].alive = jobs[j].d >= 2 && jobs[j].status == TT_OK && !jobs[j].orth_only;
  }
  std::vector<hipEvent_t> out_done(maxd, nullptr);
  hipEvent_t last_side = nullptr;
  // The output cores of step k go to the side stream once the main stream's next step has
  // been issued: nothing on the critical path reads them, so the next step starts sooner.
  struct PendingOut {
    int k = -1;
    hipEvent_t ready = nullptr;
    std::vector<std::vector<ApplyLevel>> plans;
  } pend;
  auto flush_out = [&]() -> tt_status {
    if (pend.k < 0) return TT_OK;
    hipStream_t side = side_stream(c);
    hipEvent_t done = dep_event(c);
    if (!side || !done) return fail(c, TT_EDEVICE, "side stream");
    hipError_t e2;
    if ((e2 = hipStreamWaitEvent(side, pend.ready, 0)) != hipSuccess) return hip_fail(c, e2, "event");
    c->upload_stream = side;
    tt_status r2 = launch_apply_plans(c, pend.plans, dtype, side);
    c->upload_stream = nullptr;
    if (r2 != TT_OK) return r2;
    if ((e2 = hipEventRecord(done, side)) != hipSuccess) return hip_fail(c, e2, "event");
    out_done[pend.k] = done;
    last_side = done;
    pend.k = -1;
    pend.plans.clear();
    return TT_OK;
  };
  for (int k = 0; k + 1 < maxd; ++k) {
    std::vector<int> act;
    for (int j = 0; j < nj; ++j)
      if (st[j].alive && k + 1 < jobs[j].d) act.push_back(j);
    if (act.empty()) break;
    // (1) C_k = Q_k [W_k^T; 0]: a GEMM with the explicit Q_k where it was formed, else the tree
    if (k >= 1) {
      std::vector<std::vector<ApplyLevel>> plans;
      std::vector<GemmSTask> xg;
      int xm = 0, xn = 0;
      std::vector<hipEvent_t> waited;
      for (int j : act) {
        RJob& jb = jobs[j];
        JobState& js = st[j];
        if (js.Qx[k]) {
          hipEvent_t ev = qx_done[jb.d - 1 - k];
          if (ev && std::find(waited.begin(), waited.end(), ev) == waited.end()) {
            if ((e = hipStreamWaitEvent(s, ev, 0)) != hipSuccess) return hip_fail(c, e, "event");
            waited.push_back(ev);
          }
          GemmSTask g;
          const int64_t M = jb.n[k] * js.s[k + 1], sk = js.s[k];
          g.A = js.Qx[k];   // M x s_k row-major
          g.a_rs = sk;
          g.a_cs = 1;
          g.B = js.wt;
          g.b_rs = js.t[k];
          g.b_cs = 1;
          g.C = js.C;
          g.c_rs = 1;
          g.c_cs = M;
          g.M = (int32_t)M;
          g.N = (int32_t)js.t[k];
          g.K = (int32_t)sk;
          xg.push_back(g);
          xm = std::max(xm, g.M);
          xn = std::max(xn, g.N);
          continue;
        }
        Carver cv;
        cv.base = js.ap_block;
        cv.cap = js.ap_cap;
        std::vector<ApplyLevel> pl;
        plan_apply(cv, js.rl[k], js.wt, js.t[k], js.t[k], js.C, jb.dtype, 1, jb.n[k] * js.s[k + 1], pl);
        if (cv.off > cv.cap) return fail(c, TT_ECAPACITY, "apply scratch");
        plans.push_back(std::move(pl));
      }
      tt_status rs = launch_apply_plans(c, plans, dtype);
      if (rs != TT_OK) return rs;
      if (!xg.empty()) {
        const GemmSTask* dxg = upload(c, xg);
        if (!dxg) return fail(c, TT_ENOMEM, "task upload");
        double fl = 0.0, by = 0.0;
        for (const GemmSTask& g : xg) {
          fl += 2.0 * g.M * g.N * (double)g.K;
          by += (double)elt * ((double)g.M * g.K + (double)g.M * g.N) + 8.0 * g.K * g.N;
        }
        const int pr = prof_begin(c, PK_GEMM, fl, by);
        e = launch_gemm_strided(dtype, dxg, (int)xg.size(), xm, xn, s);
        prof_end(c, pr);
        if (e != hipSuccess) return hip_fail(c, e, "explicit-Q contraction");
      }
    }
    {
      tt_status fs = flush_out();   // output cores of the previous step
      if (fs != TT_OK) return fs;
    }
    // (2) TSQR of L(C_k), into the tree block of this step's parity once the output
    // core of step k-2 (side stream) no longer reads it
    if (k >= 2 && out_done[k - 2] && (e = hipStreamWaitEvent(s, out_done[k - 2], 0)) != hipSuccess)
      return hip_fail(c, e, "event");
    std::vector<Tree*> trees;
    for (int j : act) {
      RJob& jb = jobs[j];
      JobState& js = st[j];
      Carver cv;
      cv.base = js.lr_blk[k & 1];
      cv.cap = js.lr_cap;
      std::string why;
      const int64_t M = js.t[k] * jb.n[k], N = js.s[k + 1];
      if (std::min(M, N) > SVD_BIG_MAX)
        return fail(c, TT_ENOTIMPL, "SVD of a " + std::to_string(std::min(M, N)) + "-row R factor exceeds " +
                                        std::to_string(SVD_BIG_MAX));
      if (c->autotune && !tuned_shape(M, N, jb.dtype, nullptr)) {
        tt_status ts = tune_tree(c, M, N, jb.dtype, nullptr);
        if (ts != TT_OK) return ts;
      }
      if (!plan_tree(cv, js.lr[k & 1], M, N, jb.dtype, js.C, N, 1, &why)) return fail(c, TT_ENOTIMPL, why);
      if (cv.off > cv.cap) return fail(c, TT_ECAPACITY, "left-to-right tree block");
      trees.push_back(&js.lr[k & 1]);
    }
    tt_status rs = launch_levels_factor(c, trees);
    if (rs != TT_OK) return rs;
    // (3) SVD + rank
    std::vector<SvdTask> sv;
    for (int j : act) {
      RJob& jb = jobs[j];
      JobState& js = st[j];
      SvdTask t;
      std::memset(&t, 0, sizeof(t));
      const Tree& LR = js.lr[k & 1];
      t.R = LR.root_R();
      t.r_ld = LR.rld();
      t.r_f32 = LR.root_f32();
      t.kr = LR.kr();
      t.ncol = (int32_t)LR.N;
      t.upper = 1;
      t.bulk_u = (jb.dtype == TT_F64) ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
      t.A = js.A;
      t.acc = js.acc;
      t.sigma = js.sig;
      t.perm = js.perm;
      t.iscr = js.iscr;
      t.block = (t.kr > std::min<int>(c->svd_block_min, SVD_SMALL_MAX)) ? 1 : 0;
      t.norm = js.d_norm;
      t.delta_scaled = jb.delta / std::sqrt((double)(jb.d - 1));
      // FP32-bulk: singular values below the FP32 resolution of the merged core
      // (the set-aside level 2 sqrt(s) u_32 ||x||) are noise, never kept
      t.eps_floor = (jb.dtype == TT_F32) ? fp32_eps_floor(LR.N) : 0.0;
      t.max_rank = jb.max_rank;
      t.rank_out = d_ranks + (size_t)j * (TT_MAXD + 1) + (k + 1);
      t.wt = js.wt;
      t.ur = js.urb[k & 1];
      t.t_ld = bp ? (int32_t)js.tb[k + 1] : 0;
      t.info = nullptr;
      sv.push_back(t);
    }
    const SvdTask* dsv = upload(c, sv);
    if (!sv.empty() && !dsv) return fail(c, TT_ENOMEM, "task upload");
    double sfl = 0.0, sby = 0.0;
    for (const SvdTask& t : sv) {
      const double mn = std::min(t.kr, t.ncol), mx = std::max(t.kr, t.ncol);
      sfl += 4.0 * mx * mn * mn + 22.0 * mn * mn * mn;   // R-SVD operation count (Golub-Van Loan)
      sby += 8.0 * (double)t.kr * t.ncol;
    }
    int max_kr = 0;
    for (const SvdTask& t : sv)
      if (t.block) max_kr = std::max(max_kr, (int)t.kr);
    const int spr = prof_begin(c, PK_SVD, sfl, sby);
    e = launch_svd(dsv, (int)sv.size(), s);
    if (e != hipSuccess) return hip_fail(c, e, "svd");
    if (max_kr > 0 && (e = launch_svd_big(dsv, (int)sv.size(), max_kr, s)) != hipSuccess) return hip_fail(c, e, "svd");
    prof_end(c, spr);
    if (!bp && (e = hipMemcpyAsync(h_ranks, d_ranks, (size_t)nj * (TT_MAXD + 1) * 4, hipMemcpyDeviceToHost, s)) !=
                   hipSuccess)
      return hip_fail(c, e, "rank readback");
    // rk_ev marks the U factors and trees of this step as ready for the side stream
    hipEvent_t rk_ev = dep_event(c);
    if (!rk_ev) return fail(c, TT_EDEVICE, "event");
    if ((e = hipEventRecord(rk_ev, s)) != hipSuccess) return hip_fail(c, e, "event");
    if (!bp && (e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "sync");
    // (4) output core k = Q_M [U_t; 0]
    std::vector<std::vector<ApplyLevel>> plans;
    for (int j : act) {
      RJob& jb = jobs[j];
      JobState& js = st[j];
      const int64_t tk1 = bp ? js.tb[k + 1] : h_ranks[(size_t)j * (TT_MAXD + 1) + (k + 1)];
      if (tk1 < 1 || tk1 > js.tb[k + 1]) return fail(c, TT_EDEVICE, "rank out of range");
      js.t[k + 1] = tk1;
      const int64_t sz = js.t[k] * jb.n[k] * tk1;
      if (!bp && js.out_off + sz > jb.out->capacity) {
        jb.status = TT_ECAPACITY;
        js.alive = false;
        continue;
      }
      // at the bounds the core goes to its staging slot, compacted at the end
      char* dst = bp ? js.stage + (size_t)js.stg_off[k] * elt : (char*)jb.out->data + (size_t)js.out_off * elt;
      Carver cv;
      cv.base = js.ap_side;
      cv.cap = js.ap_cap;
      std::vector<ApplyLevel> pl;
      plan_apply(cv, js.lr[k & 1], js.urb[k & 1], tk1, tk1, dst, jb.dtype, tk1, 1, pl);
      if (cv.off > cv.cap) return fail(c, TT_ECAPACITY, "apply scratch");
      plans.push_back(std::move(pl));
      js.out_off += sz;
    }
    // on the side stream, after the next step's first launch: the next step only needs W
    // (already final), not this core
    if (!plans.empty()) {
      pend.k = k;
      pend.ready = rk_ev;
      pend.plans = std::move(plans);
      // with many jobs the side stream carries as much work as the main one and planning the
      // next step takes long: launch the output cores now
      if (act.size() > 4 || bp) {
        tt_status fs = flush_out();
        if (fs != TT_OK) return fs;
      }
    }
  }
  {
    tt_status fs = flush_out();
    if (fs != TT_OK) return fs;
  }
  // the output cores written on the side stream are complete before anything reads them
  if (last_side && (e = hipStreamWaitEvent(s, last_side, 0)) != hipSuccess) return hip_fail(c, e, "event");
  // ---------------- last core
  {
    std::vector<std::vector<ApplyLevel>> plans;
    for (int j = 0; j < nj; ++j) {
      RJob& jb = jobs[j];
      JobState& js = st[j];
      if (!js.alive) continue;
      const int k = jb.d - 1;
      const int64_t sz = js.t[k] * jb.n[k];
      if (!bp && js.out_off + sz > jb.out->capacity) {
        jb.status = TT_ECAPACITY;
        js.alive = false;
        continue;
      }
      char* dst = bp ? js.stage + (size_t)js.stg_off[k] * elt : (char*)jb.out->data + (size_t)js.out_off * elt;
      Carver cv;
      cv.base = js.ap_block;
      cv.cap = js.ap_cap;
      std::vector<ApplyLevel> pl;
      plan_apply(cv, js.rl[k], js.wt, js.t[k], js.t[k], dst, jb.dtype, 1, jb.n[k], pl);
      if (cv.off > cv.cap) return fail(c, TT_ECAPACITY, "apply scratch");
      plans.push_back(std::move(pl));
      js.out_off += sz;
    }
    tt_status rs = launch_apply_plans(c, plans, dtype);
    if (rs != TT_OK) return rs;
  }
  if (bp) {
    // ---------------- cores from their bound shapes into the packed results, at the device's ranks
    std::vector<int32_t> hst(nj);
    std::vector<int64_t> geo;
    std::vector<size_t> goff(nj, 0);
    for (int j = 0; j < nj; ++j) {
      const RJob& jb = jobs[j];
      hst[j] = (int32_t)jb.status;
      if (jb.d < 2 || jb.orth_only || !st[j].alive) continue;
      goff[j] = geo.size();
      for (int k = 0; k < jb.d; ++k) geo.push_back(jb.n[k]);
      for (int k = 0; k <= jb.d; ++k) geo.push_back(st[j].tb[k]);
      for (int k = 0; k < jb.d; ++k) geo.push_back(st[j].stg_off[k]);
    }
    int32_t* d_status = (int32_t*)dev_scratch(c, (size_t)nj * 4);   // written by the compaction
    const int64_t* dgeo = geo.empty() ? nullptr : upload(c, geo);
    if (!d_status || (!geo.empty() && !dgeo)) return fail(c, TT_ENOMEM, "compaction buffers");
    std::vector<CompactTask> ct;
    for (int j = 0; j < nj; ++j) {
      const RJob& jb = jobs[j];
      CompactTask t;
      std::memset(&t, 0, sizeof(t));
      t.d = jb.d;
      t.ranks = d_ranks + (size_t)j * (TT_MAXD + 1);
      t.status = d_status + j;
      t.init_status = hst[j];   // the status decided on the host; the compaction may add TT_ECAPACITY
      t.active = (jb.d >= 2 && !jb.orth_only && st[j].alive && jb.status == TT_OK) ? 1 : 0;
      if (t.active) {
        t.staging = st[j].stage;
        t.out = jb.out->data;
        t.capacity = jb.out->capacity;
        t.geo = dgeo + goff[j];
      }
      ct.push_back(t);
    }
    const CompactTask* dct = upload(c, ct);
    if (!dct) return fail(c, TT_ENOMEM, "task upload");
    if ((e = launch_compact(dtype, dct, (int)ct.size(), s)) != hipSuccess) return hip_fail(c, e, "compaction");
    if (mode.async) {
      // results, ranks, statuses and norms reach the caller through copies on the stream
      if ((e = hipMemcpyAsync(mode.ranks, d_ranks, (size_t)nj * (TT_MAXD + 1) * 4, hipMemcpyDeviceToHost, s)) !=
              hipSuccess ||
          (e = hipMemcpyAsync(mode.status, d_status, (size_t)nj * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
          (mode.norms && (e = hipMemcpyAsync(mode.norms, d_norms, (size_t)nj * 8, hipMemcpyDeviceToHost, s)) !=
                             hipSuccess))
        return hip_fail(c, e, "result copies");
      return TT_OK;
    }
    int32_t* h_status = (int32_t*)c->pin.alloc((size_t)nj * 4);
    if (!h_status) return fail(c, TT_ENOMEM, "small buffers");
    if ((e = hipMemcpyAsync(h_ranks, d_ranks, (size_t)nj * (TT_MAXD + 1) * 4, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(h_status, d_status, (size_t)nj * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
      return hip_fail(c, e, "rank readback");
    if ((e = hipMemcpyAsync(h_norms, d_norms, (size_t)nj * 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
      return hip_fail(c, e, "norm readback");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "sync");
    for (int j = 0; j < nj; ++j) {
      RJob& jb = jobs[j];
      jb.status = (tt_status)h_status[j];
      if (jb.status != TT_OK) continue;
      jb.norm = h_norms[j];
      if (jb.orth_only) continue;
      for (int k = 0; k <= jb.d; ++k) jb.out->r[k] = h_ranks[(size_t)j * (TT_MAXD + 1) + k];
    }
    return TT_OK;
  }
  // ---------------- norms back, ranks out
  if ((e = hipMemcpyAsync(h_norms, d_norms, (size_t)nj * 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(c, e, "norm readback");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "sync");
  for (int j = 0; j < nj; ++j) {
    RJob& jb = jobs[j];
    if (jb.status != TT_OK) continue;
    jb.norm = h_norms[j];
    if (jb.orth_only) continue;
    if (jb.d == 1) {
      jb.out->r[0] = 1;
      jb.out->r[1] = 1;
      continue;
    }
    jb.out->r[0] = 1;
    for (int k = 1; k < jb.d; ++k) jb.out->r[k] = st[j].t[k];
    jb.out->r[jb.d] = 1;
  }
  return TT_OK;
}

// ============================================================================
// Randomized rounding of a lazy sum (Randomize-then-Orthogonalize, FP64).
//   W_k = cores k..d-1 of x contracted with those of the sketch (R_k x l_k),
//         right to left, per sum component (block rows of W_k);
//   left to right, core k = 0..d-2:
//     Z_k = L(G_k) W_{k+1};  Z_k = Q R (tile QR tree);  core k of the result = Q
//     M_k = Q^T L(G_k);      G_{k+1} = M_k x_1 core k+1 (per component block)
//   last core = G_{d-1};  with delta > 0 the result is rounded deterministically.
// G_0 is the side-by-side first core with the sum coefficients; the last core
// stacks the components' last cores.  Every product is a strided GEMM.
// ============================================================================
namespace {

struct Gemms {
  std::vector<GemmSTask> t;
  int max_m = 0, max_n = 0;
  void add(const void* A, int64_t a_rs, int64_t a_cs, const double* B, int64_t b_rs, int64_t b_cs, void* C,
           int64_t c_rs, int64_t c_cs, int64_t M, int64_t N, int64_t K) {
    if (M <= 0 || N <= 0) return;
    GemmSTask g;
    std::memset(&g, 0, sizeof(g));
    g.A = A;
    g.a_rs = a_rs;
    g.a_cs = a_cs;
    g.B = B;
    g.b_rs = b_rs;
    g.b_cs = b_cs;
    g.C = C;
    g.c_rs = c_rs;
    g.c_cs = c_cs;
    g.M = (int32_t)M;
    g.N = (int32_t)N;
    g.K = (int32_t)K;
    t.push_back(g);
    max_m = std::max<int>(max_m, (int)M);
    max_n = std::max<int>(max_n, (int)N);
  }
  tt_status run(tt_ctx* c) {
    if (t.empty()) return TT_OK;
    const GemmSTask* dt = upload(c, t);
    if (!dt) return fail(c, TT_ENOMEM, "gemm task upload");
    double fl = 0.0;
    if (c->prof)
      for (const auto& g : t) fl += 2.0 * g.M * g.N * (double)g.K;
    const int pr = prof_begin(c, PK_GEMM, fl, 0.0);
    hipError_t e = launch_gemm_strided(TT_F64, dt, (int)t.size(), max_m, max_n, c->stream);
    prof_end(c, pr);
    if (e != hipSuccess) return hip_fail(c, e, "gemm");
    t.clear();
    max_m = max_n = 0;
    return TT_OK;
  }
};

tt_status run_copies(tt_ctx* c, const std::vector<CopySeg>& segs) {
  if (segs.empty()) return TT_OK;
  const CopySeg* ds = upload(c, segs);
  if (!ds) return fail(c, TT_ENOMEM, "copy upload");
  hipError_t e = launch_copy_segs(TT_F64, ds, (int)segs.size(), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "copy");
  return TT_OK;
}

}  // namespace

tt_status round_randomized(tt_ctx* c, const tt_sum* x, const tt_vec* sk, double delta, tt_vec* out) {
  RJob jb;
  make_job(c, x, 0.0, 0, nullptr, jb);
  const int d = jb.d;
  const int nc = (int)jb.comps.size();
  const int64_t* n = jb.n;
  const int64_t* R = jb.R;
  const size_t mark = c->ws_off;
  struct Mark {
    tt_ctx* c;
    size_t off;
    ~Mark() { c->ws_off = off; }
  } wmark{c, mark};
  c->ws_overflow = false;
  int64_t l[TT_MAXD + 1], p[TT_MAXD + 1];
  for (int k = 0; k <= d; ++k) l[k] = sk->r[k];
  p[0] = p[d] = 1;
  for (int k = 1; k < d; ++k) p[k] = std::min<int64_t>(l[k], p[k - 1] * n[k - 1]);
  auto roff = [&](int ci, int k) { return jb.roff[(size_t)ci * (d + 1) + k]; };
  auto core = [&](int ci, int k) { return (const double*)jb.comps[ci].data + jb.comps[ci].core_off[k]; };
  auto rc = [&](int ci, int k) { return jb.comps[ci].r[k]; };
  // FP32 storage: the components are converted to FP64 in the workspace, the sweep runs in
  // FP64 and its result is converted back before the rounding at delta (FP32-bulk)
  const bool f32 = (jb.dtype == TT_F32);
  if (f32) {
    for (int ci = 0; ci < nc; ++ci) {
      int64_t sz = 0;
      for (int k = 0; k < d; ++k) sz += rc(ci, k) * n[k] * rc(ci, k + 1);
      double* cp = (double*)ws_alloc(c, (size_t)sz * 8);
      if (!cp) return fail(c, TT_ECAPACITY, "workspace too small for randomized rounding: need " + std::to_string(c->required));
      hipError_t ce = launch_cast(TT_F32, jb.comps[ci].data, TT_F64, cp, sz, c->stream);
      if (ce != hipSuccess) return hip_fail(c, ce, "cast");
      jb.comps[ci].data = (const char*)cp;
    }
  }
  // sketch cores
  const double* S[TT_MAXD];
  {
    int64_t off = 0;
    for (int k = 0; k < d; ++k) {
      S[k] = (const double*)sk->data + off;
      off += sk->r[k] * sk->n[k] * sk->r[k + 1];
    }
  }
  // ---- buffers (workspace)
  Carver ws;
  ws.ctx = c;
  double* WT[TT_MAXD + 1] = {nullptr};
  size_t t1max = 1, gmax = 1, zmax = 1, mmax = 1, pmax = 1;
  for (int k = 1; k < d; ++k) WT[k] = (double*)ws.take((size_t)l[k] * R[k] * 8);
  for (int k = 1; k + 1 < d; ++k) t1max = std::max<size_t>(t1max, (size_t)(R[k] * n[k] * l[k + 1]));
  for (int k = 0; k + 1 < d; ++k) {
    gmax = std::max<size_t>(gmax, (size_t)(p[k] * n[k] * R[k + 1]));
    zmax = std::max<size_t>(zmax, (size_t)(p[k] * n[k] * l[k + 1]));
    mmax = std::max<size_t>(mmax, (size_t)(p[k + 1] * R[k + 1]));
    pmax = std::max<size_t>(pmax, (size_t)p[k + 1]);
  }
  double* T1 = (double*)ws.take(t1max * 8);
  double* Gb[2] = {(double*)ws.take(gmax * 8), (double*)ws.take(gmax * 8)};
  double* Z = (double*)ws.take(zmax * 8);
  double* Mb = (double*)ws.take(mmax * 8);
  double* Xs = (double*)ws.take((size_t)(R[d - 1] * n[d - 1]) * 8);
  double* eye = (double*)ws.take(pmax * pmax * 8);
  int64_t need = 0;
  for (int k = 0; k < d; ++k) need += p[k] * n[k] * p[k + 1];
  tt_vec res = *out;
  res.dtype = TT_F64;
  for (int k = 0; k <= d; ++k) res.r[k] = p[k];
  void* res32 = nullptr;   // FP32 copy of the result, rounded at delta into out
  if (delta > 0.0 || f32) {
    res.data = ws.take((size_t)need * 8);
    res.capacity = need;
    if (f32 && delta > 0.0) res32 = ws.take((size_t)need * 4);
    if ((f32 && delta > 0.0 && !res32))
      return fail(c, TT_ECAPACITY, "workspace too small for randomized rounding: need " + std::to_string(c->required));
  }
  if (delta <= 0.0 && out->capacity < need) {
    return fail(c, TT_ECAPACITY, "randomized rounding: out capacity " + std::to_string(out->capacity) + " < " +
                                     std::to_string(need));
  }
  if (c->ws_overflow || !T1 || !Gb[0] || !Gb[1] || !Z || !Mb || !Xs || !eye || ((delta > 0.0 || f32) && !res.data))
    return fail(c, TT_ECAPACITY, "workspace too small for randomized rounding: need " + std::to_string(c->required));
  for (int k = 1; k < d; ++k)
    if (!WT[k]) return fail(c, TT_ECAPACITY, "workspace too small for randomized rounding");
  tt_status s;
  hipError_t e;
  // ---- sketch contractions, right to left: WT_k (l_k x R_k), block columns per component
  Gemms gm;
  for (int k = d - 1; k >= 1; --k) {
    // T1^c = L(X^c_k) W^c_{k+1}  ((r^c_k n_k) x l_{k+1}); for k = d-1, W_d = 1 and T1^c = X^c_{d-1}
    std::vector<const double*> t1(nc);
    if (k + 1 < d) {
      int64_t off = 0;
      for (int ci = 0; ci < nc; ++ci) {
        t1[ci] = T1 + off;
        gm.add(core(ci, k), rc(ci, k + 1), 1, WT[k + 1] + roff(ci, k + 1), 1, R[k + 1], T1 + off, l[k + 1], 1,
               rc(ci, k) * n[k], l[k + 1], rc(ci, k + 1));
        off += rc(ci, k) * n[k] * l[k + 1];
      }
      if ((s = gm.run(c)) != TT_OK) return s;
    } else {
      for (int ci = 0; ci < nc; ++ci) t1[ci] = core(ci, k);
    }
    // WT_k[j][roff + a] = sum_q T1^c[a][q] S_k[j][q]   (q over n_k l_{k+1})
    const int64_t K = n[k] * l[k + 1];
    for (int ci = 0; ci < nc; ++ci)
      gm.add(t1[ci], K, 1, S[k], 1, K, WT[k] + roff(ci, k), 1, R[k], rc(ci, k), l[k], K);
    if ((s = gm.run(c)) != TT_OK) return s;
  }
  // ---- G_0: first cores side by side, with the sum coefficients
  {
    std::vector<CopySeg> segs;
    for (int ci = 0; ci < nc; ++ci)
      for (int64_t i = 0; i < n[0]; ++i) {
        CopySeg g;
        std::memset(&g, 0, sizeof(g));
        g.src = core(ci, 0) + i * rc(ci, 1);
        g.dst = Gb[0] + i * R[1] + roff(ci, 1);
        g.count = rc(ci, 1);
        g.coef = jb.comps[ci].coef;
        segs.push_back(g);
      }
    if ((s = run_copies(c, segs)) != TT_OK) return s;
  }
  // ---- left to right
  int64_t ooff = 0;
  for (int k = 0; k + 1 < d; ++k) {
    double* G = Gb[k & 1];
    double* Gn = Gb[(k + 1) & 1];
    const int64_t Mz = p[k] * n[k];
    // Z = L(G_k) W_{k+1}
    gm.add(G, R[k + 1], 1, WT[k + 1], 1, R[k + 1], Z, l[k + 1], 1, Mz, l[k + 1], R[k + 1]);
    if ((s = gm.run(c)) != TT_OK) return s;
    // Q of Z: tile QR tree, then Q [I; 0] into core k of the result
    Tree tree;
    std::string why;
    if (!plan_tree(ws, tree, Mz, l[k + 1], TT_F64, Z, l[k + 1], 1, &why))
      return fail(c, c->ws_overflow ? TT_ECAPACITY : TT_ENOTIMPL, "randomized rounding: " + why);
    if (c->ws_overflow)   // a tile or T buffer of the tree did not fit: launch nothing
      return fail(c, TT_ECAPACITY, "workspace too small for randomized rounding: need " + std::to_string(c->required));
    if (tree.kr() != p[k + 1]) return fail(c, TT_EINVAL, "randomized rounding: unexpected rank of Z");
    std::vector<Tree*> trees{&tree};
    if ((s = launch_levels_factor(c, trees)) != TT_OK) return s;
    if ((e = launch_eye(eye, (int)p[k + 1], c->stream)) != hipSuccess) return hip_fail(c, e, "eye");
    double* Qk = (double*)res.data + ooff;
    std::vector<std::vector<ApplyLevel>> plans(1);
    plan_apply(ws, tree, eye, p[k + 1], p[k + 1], Qk, TT_F64, p[k + 1], 1, plans[0]);
    if (c->ws_overflow) return fail(c, TT_ECAPACITY, "workspace too small for randomized rounding: need " +
                                                         std::to_string(c->required));
    if ((s = launch_apply_plans(c, plans, TT_F64)) != TT_OK) return s;
    ooff += Mz * p[k + 1];
    // M = Q^T L(G_k)   (p_{k+1} x R_{k+1})
    gm.add(Qk, 1, p[k + 1], G, R[k + 1], 1, Mb, R[k + 1], 1, p[k + 1], R[k + 1], Mz);
    if ((s = gm.run(c)) != TT_OK) return s;
    if (k + 2 < d) {
      // G_{k+1}[a][i][roff_c + b] = sum_b' M[a][roff'_c + b'] X^c_{k+1}[b'][i][b]
      for (int ci = 0; ci < nc; ++ci)
        for (int64_t i = 0; i < n[k + 1]; ++i)
          gm.add(Mb + roff(ci, k + 1), R[k + 1], 1, core(ci, k + 1) + i * rc(ci, k + 2), n[k + 1] * rc(ci, k + 2), 1,
                 Gn + i * R[k + 2] + roff(ci, k + 2), n[k + 1] * R[k + 2], 1, p[k + 1], rc(ci, k + 2), rc(ci, k + 1));
      if ((s = gm.run(c)) != TT_OK) return s;
    } else {
      // last core: the components' last cores stacked, then M times the stack
      std::vector<CopySeg> segs;
      for (int ci = 0; ci < nc; ++ci) {
        CopySeg g;
        std::memset(&g, 0, sizeof(g));
        g.src = core(ci, d - 1);
        g.dst = Xs + roff(ci, d - 1) * n[d - 1];
        g.count = rc(ci, d - 1) * n[d - 1];
        g.coef = 1.0;
        segs.push_back(g);
      }
      if ((s = run_copies(c, segs)) != TT_OK) return s;
      gm.add(Mb, R[d - 1], 1, Xs, n[d - 1], 1, (double*)res.data + ooff, n[d - 1], 1, p[d - 1], n[d - 1], R[d - 1]);
      if ((s = gm.run(c)) != TT_OK) return s;
    }
  }
  tt_vec fin = res;   // the result in the storage precision
  if (f32) {
    fin.dtype = TT_F32;
    fin.data = (delta > 0.0) ? res32 : out->data;
    if ((e = launch_cast(TT_F64, res.data, TT_F32, fin.data, need, c->stream)) != hipSuccess) return hip_fail(c, e, "cast");
  }
  if (delta > 0.0) {
    static const double one = 1.0;
    tt_sum rs{1, &one, &fin};
    std::vector<RJob> jobs(1);
    make_job(c, &rs, delta, 0, out, jobs[0]);
    if ((s = round_jobs(c, jobs)) != TT_OK) return s;
    if (jobs[0].status != TT_OK) return fail(c, jobs[0].status, "randomized rounding: output capacity");
  } else {
    for (int k = 0; k <= d; ++k) out->r[k] = p[k];
  }
  return TT_OK;
}

}  // namespace tto
