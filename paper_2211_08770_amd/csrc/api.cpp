// extern "C" entry points of libttortho: argument checking, buffer planning
// and the sequencing of the orthogonalization schemes (Algorithms 1-5 of the
// paper).  All arithmetic on TT data and on the small FP64 matrices runs in
// the kernels; this file only decides what to launch and moves descriptors,
// ranks and scalar coefficients between host and device.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "host.h"

using namespace tto;

// ============================================================================
// arenas, workspace, errors
// ============================================================================
namespace tto {

char* Arena::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (chunks.empty() || off + bytes > chunks.back().second) {
    size_t want = std::max<size_t>(bytes, chunks.empty() ? (size_t)4 << 20 : chunks.back().second * 2);
    char* p = nullptr;
    hipError_t e = pinned ? hipHostMalloc((void**)&p, want, hipHostMallocDefault) : hipMalloc((void**)&p, want);
    if (e != hipSuccess || !p) return nullptr;
    chunks.push_back({p, want});
    off = 0;
  }
  char* p = chunks.back().first + off;
  off += bytes;
  used_total += bytes;
  return p;
}

void Arena::reset() {
  // keep one chunk big enough for the whole of the last call
  if (chunks.size() > 1) {
    size_t total = 0;
    for (auto& c : chunks) total += c.second;
    release();
    char* p = nullptr;
    hipError_t e = pinned ? hipHostMalloc((void**)&p, total, hipHostMallocDefault) : hipMalloc((void**)&p, total);
    if (e == hipSuccess && p) chunks.push_back({p, total});
  }
  off = 0;
  used_total = 0;
}

void Arena::release() {
  for (auto& c : chunks) {
    if (pinned) (void)hipHostFree(c.first);
    else (void)hipFree(c.first);
  }
  chunks.clear();
  off = 0;
}

tt_status fail(tt_ctx* c, tt_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

tt_status hip_fail(tt_ctx* c, hipError_t e, const char* where) {
  return fail(c, TT_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

void* ws_alloc(tt_ctx* c, size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  const size_t off = c->ws_off;
  c->ws_off += bytes;
  c->required = std::max(c->required, c->ws_off);
  if (c->ws_off > c->ws_bytes || c->ws == nullptr) {
    c->ws_overflow = true;
    return nullptr;
  }
  return c->ws + off;
}

char* ReplayArena::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  while (cur < chunks.size() && off + bytes > chunks[cur].second) {
    ++cur;
    off = 0;
  }
  if (cur == chunks.size()) {
    const size_t want = std::max<size_t>(bytes, chunks.empty() ? (size_t)1 << 20 : chunks.back().second * 2);
    char* p = nullptr;
    if (hipMalloc((void**)&p, want) != hipSuccess || !p) return nullptr;
    chunks.push_back({p, want});
    off = 0;
  }
  char* p = chunks[cur].first + off;
  off += bytes;
  return p;
}

void ReplayArena::release() {
  for (auto& ch : chunks) (void)hipFree(ch.first);
  chunks.clear();
  rewind();
}

void* upload_bytes(tt_ctx* c, const void* src, size_t bytes) {
  if (c->graph_arena) {
    char* d = c->graph_arena->alloc(bytes);
    if (!d) return nullptr;
    if (c->graph_capturing) return d;   // the building pass put the same bytes here
    char* h = c->pin.alloc(bytes);
    if (!h) return nullptr;
    std::memcpy(h, src, bytes);
    if (hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c->upload_stream ? c->upload_stream : c->stream) !=
        hipSuccess)
      return nullptr;
    return d;
  }
  char* d = c->dev.alloc(bytes);
  char* h = c->pin.alloc(bytes);
  if (!d || !h) return nullptr;
  std::memcpy(h, src, bytes);
  if (hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c->upload_stream ? c->upload_stream : c->stream) !=
      hipSuccess)
    return nullptr;
  return d;
}

void* dev_scratch(tt_ctx* c, size_t bytes) { return c->graph_arena ? c->graph_arena->alloc(bytes) : c->dev.alloc(bytes); }

static hipEvent_t prof_event(tt_ctx* c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

hipStream_t side_stream(tt_ctx* c) {
  if (!c->side && hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) c->side = nullptr;
  return c->side;
}

hipEvent_t dep_event(tt_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

int prof_begin(tt_ctx* c, int kind, double flops, double bytes, hipStream_t s) {
  if (!c->prof) return -1;
  if (!s) s = c->stream;
  ProfRec r;
  r.kind = kind;
  r.flops = flops;
  r.bytes = bytes;
  r.start = prof_event(c);
  r.stop = prof_event(c);
  if (!r.start || !r.stop) return -1;
  if (hipEventRecord(r.start, s) != hipSuccess) return -1;
  c->prof_open.push_back(r);
  return (int)c->prof_open.size() - 1;
}

void prof_end(tt_ctx* c, int rec, hipStream_t s) {
  if (rec < 0 || !c->prof) return;
  (void)hipEventRecord(c->prof_open[rec].stop, s ? s : c->stream);
}

void prof_collect(tt_ctx* c) {
  for (ProfRec& r : c->prof_open) {
    float ms = 0.f;
    if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      c->prof_ms[r.kind] += ms;
      c->prof_flops[r.kind] += r.flops;
      c->prof_bytes[r.kind] += r.bytes;
      c->prof_cnt[r.kind] += 1;
    }
    c->prof_pool.push_back(r.start);
    c->prof_pool.push_back(r.stop);
  }
  c->prof_open.clear();
}

}  // namespace tto

namespace {

// Resets the per-call arenas once the stream has drained (every entry point
// synchronises before returning, so nothing in flight refers to them).
// Wait for the last asynchronous call of the context (its copies may still read
// the staging arenas and its kernels the workspace).
void wait_async(tt_ctx* c) {
  if (c->async_pending) {
    (void)hipEventSynchronize(c->async_done);
    c->async_pending = false;
  }
}

struct CallScope {
  tt_ctx* c;
  bool async = false;   // leave the work in flight: record async_done instead of draining the streams
  explicit CallScope(tt_ctx* ctx) : c(ctx) {
    c->err.clear();
    (void)hipSetDevice(c->device);
    wait_async(c);
  }
  ~CallScope() {
    if (async && c->async_done && hipEventRecord(c->async_done, c->stream) == hipSuccess) {
      c->async_pending = true;
    } else {
      if (c->side) (void)hipStreamSynchronize(c->side);
      (void)hipStreamSynchronize(c->stream);
      prof_collect(c);
    }
    c->ev_used = 0;
    c->dev.reset();
    c->pin.reset();
  }
};

int64_t packed_size(const tt_vec* v) {
  int64_t s = 0;
  for (int k = 0; k < v->d; ++k) s += v->r[k] * v->n[k] * v->r[k + 1];
  return s;
}

tt_status check_vec(tt_ctx* c, const tt_vec* v, const char* what, bool input) {
  if (!v) return fail(c, TT_EINVAL, std::string(what) + ": null tt_vec");
  if (v->d < 1 || v->d > TT_MAXD) return fail(c, TT_EINVAL, std::string(what) + ": order d out of [1, 64]");
  if (v->dtype != TT_F64 && v->dtype != TT_F32) return fail(c, TT_EINVAL, std::string(what) + ": bad dtype");
  for (int k = 0; k < v->d; ++k)
    if (v->n[k] < 1) return fail(c, TT_EINVAL, std::string(what) + ": mode size < 1");
  if (!v->data) return fail(c, TT_EINVAL, std::string(what) + ": null data");
  if (input) {
    if (v->r[0] != 1 || v->r[v->d] != 1) return fail(c, TT_EINVAL, std::string(what) + ": r_0 and r_d must be 1");
    for (int k = 1; k < v->d; ++k)
      if (v->r[k] < 1) return fail(c, TT_EINVAL, std::string(what) + ": rank < 1");
    if (v->capacity < packed_size(v))
      return fail(c, TT_EINVAL, std::string(what) + ": capacity smaller than the packed cores");
  }
  return TT_OK;
}

tt_status check_sum(tt_ctx* c, const tt_sum* x, const char* what) {
  if (!x || x->ncomp < 1 || !x->comp || !x->coef)
    return fail(c, TT_EINVAL, std::string(what) + ": empty or null sum");
  tt_status s;
  for (int i = 0; i < x->ncomp; ++i) {
    if ((s = check_vec(c, &x->comp[i], what, true)) != TT_OK) return s;
    if (!std::isfinite(x->coef[i])) return fail(c, TT_EINVAL, std::string(what) + ": non-finite coefficient");
    const tt_vec& a = x->comp[0];
    const tt_vec& b = x->comp[i];
    if (a.d != b.d || a.dtype != b.dtype) return fail(c, TT_EINVAL, std::string(what) + ": components differ in d/dtype");
    for (int k = 0; k < a.d; ++k)
      if (a.n[k] != b.n[k]) return fail(c, TT_EINVAL, std::string(what) + ": components differ in mode sizes");
  }
  return TT_OK;
}

bool same_shape(const tt_vec& a, const tt_vec& b) {
  if (a.d != b.d || a.dtype != b.dtype) return false;
  for (int k = 0; k < a.d; ++k)
    if (a.n[k] != b.n[k]) return false;
  return true;
}

// caps_k = min(prod_{j<k} n_j, prod_{j>=k} n_j), saturating
void rank_caps(const tt_vec& v, int64_t* caps) {
  const int d = v.d;
  const int64_t BIG = std::numeric_limits<int64_t>::max() / 4;
  caps[0] = caps[d] = 1;
  for (int k = 1; k < d; ++k) {
    int64_t l = 1, r = 1;
    for (int j = 0; j < k; ++j) l = (l > BIG / v.n[j]) ? BIG : l * v.n[j];
    for (int j = k; j < d; ++j) r = (r > BIG / v.n[j]) ? BIG : r * v.n[j];
    caps[k] = std::min(l, r);
  }
}

}  // namespace

namespace tto {

tt_status make_job(tt_ctx* c, const tt_sum* x, double delta, int64_t max_rank, tt_vec* out, RJob& job) {
  const tt_vec& v0 = x->comp[0];
  job.d = v0.d;
  job.dtype = v0.dtype;
  for (int k = 0; k < job.d; ++k) job.n[k] = v0.n[k];
  job.comps.clear();
  job.roff.assign((size_t)x->ncomp * (job.d + 1), 0);
  for (int k = 0; k <= job.d; ++k) job.R[k] = 0;
  for (int i = 0; i < x->ncomp; ++i) {
    const tt_vec& v = x->comp[i];
    Comp cp;
    cp.data = (const char*)v.data;
    cp.coef = x->coef[i];
    int64_t off = 0;
    for (int k = 0; k <= job.d; ++k) cp.r[k] = v.r[k];
    for (int k = 0; k < job.d; ++k) {
      cp.core_off[k] = off;
      off += v.r[k] * v.n[k] * v.r[k + 1];
    }
    for (int k = 0; k <= job.d; ++k) {
      job.roff[(size_t)i * (job.d + 1) + k] = job.R[k];
      job.R[k] += v.r[k];
    }
    job.comps.push_back(cp);
  }
  job.R[0] = job.R[job.d] = 1;
  job.delta = delta;
  job.max_rank = max_rank;
  job.out = out;
  job.status = TT_OK;
  (void)c;
  return TT_OK;
}

// out_dev[p] = <xs[p], ys[p]> = sum_{c, c'} coef_c coef'_c' <x_c, y_c'>  (device doubles).
// When out_idx is given the p-th result goes to out_dev[out_idx[p]].
tt_status dot_pairs_idx(tt_ctx* c, int npairs, const tt_sum* xs, const tt_sum* ys, double* out_dev,
                        const std::vector<int32_t>* out_idx) {
  if (npairs <= 0) return TT_OK;
  const int dtype = xs[0].comp[0].dtype;
  const size_t elt = elt_size(dtype);
  struct Mark {
    tt_ctx* c;
    size_t off;
    ~Mark() { c->ws_off = off; }
  } mark{c, c->ws_off};
  // device geometry per distinct component
  std::vector<const tt_vec*> uniq;
  std::vector<int64_t> geo;
  auto geom_of = [&](const tt_vec* v) -> size_t {
    for (size_t i = 0; i < uniq.size(); ++i)
      if (uniq[i] == v) return i;
    uniq.push_back(v);
    return uniq.size() - 1;
  };
  struct Pair {
    size_t gx, gy;
    const tt_vec* x;
    const tt_vec* y;
    double coef;
    int64_t wcap, tcap;
  };
  std::vector<Pair> pairs;
  std::vector<int32_t> seg(1, 0);
  for (int p = 0; p < npairs; ++p) {
    for (int a = 0; a < xs[p].ncomp; ++a) {
      for (int b = 0; b < ys[p].ncomp; ++b) {
        const tt_vec* x = &xs[p].comp[a];
        const tt_vec* y = &ys[p].comp[b];
        if (!same_shape(*x, *y)) return fail(c, TT_EINVAL, "dot: operands differ in d, n or dtype");
        Pair pr;
        pr.x = x;
        pr.y = y;
        pr.gx = geom_of(x);
        pr.gy = geom_of(y);
        pr.coef = xs[p].coef[a] * ys[p].coef[b];
        pr.wcap = 1;
        pr.tcap = 1;
        for (int k = 0; k < x->d; ++k) {
          pr.wcap = std::max(pr.wcap, x->r[k + 1] * y->r[k + 1]);
          pr.tcap = std::max(pr.tcap, x->r[k] * x->n[k] * y->r[k + 1]);
        }
        pairs.push_back(pr);
      }
    }
    seg.push_back((int32_t)pairs.size());
  }
  // geometry upload: per component [n(d) | r(d+1)]
  std::vector<size_t> goff;
  for (const tt_vec* v : uniq) {
    goff.push_back(geo.size());
    for (int k = 0; k < v->d; ++k) geo.push_back(v->n[k]);
    for (int k = 0; k <= v->d; ++k) geo.push_back(v->r[k]);
  }
  const int64_t* dgeo = upload(c, geo);
  double* slots = (double*)dev_scratch(c, pairs.size() * 8);
  if (!dgeo || !slots) return fail(c, TT_ENOMEM, "dot buffers");
  // scratch in chunks bounded by a budget
  const size_t budget = (size_t)256 << 20;
  size_t i0 = 0;
  while (i0 < pairs.size()) {
    size_t bytes = 0, i1 = i0;
    while (i1 < pairs.size()) {
      const size_t need = ((size_t)(2 * pairs[i1].wcap + pairs[i1].tcap) * sizeof(double) + 511) & ~(size_t)255;
      if (i1 > i0 && bytes + need > budget) break;
      bytes += need;
      ++i1;
    }
    char* scratch = (char*)ws_alloc(c, bytes);
    if (!scratch) return fail(c, TT_ECAPACITY, "workspace too small for dot scratch: need " + std::to_string(c->required));
    std::vector<DotTask> tasks;
    size_t o = 0;
    for (size_t i = i0; i < i1; ++i) {
      const Pair& pr = pairs[i];
      DotTask t;
      std::memset(&t, 0, sizeof(t));
      t.d = pr.x->d;
      t.x = pr.x->data;
      t.y = pr.y->data;
      t.nn = dgeo + goff[pr.gx];
      t.rx = dgeo + goff[pr.gx] + pr.x->d;
      t.ry = dgeo + goff[pr.gy] + pr.y->d;
      t.coef = pr.coef;
      t.w = scratch + o;
      t.wcap = pr.wcap;
      o += (size_t)2 * pr.wcap * sizeof(double);   // W and tmp are FP64 in both precisions
      o = (o + 255) & ~(size_t)255;
      t.tmp = scratch + o;
      o += (size_t)pr.tcap * sizeof(double);
      o = (o + 255) & ~(size_t)255;
      t.out = slots + i;
      tasks.push_back(t);
    }
    const DotTask* dt = upload(c, tasks);
    if (!dt) return fail(c, TT_ENOMEM, "dot tasks");
    double fl = 0.0, by = 0.0;
    for (size_t i = i0; i < i1; ++i) {
      const tt_vec* x = pairs[i].x;
      const tt_vec* y = pairs[i].y;
      for (int k = 0; k < x->d; ++k) {
        fl += 2.0 * x->r[k] * x->n[k] * y->r[k + 1] * (double)(y->r[k] + x->r[k + 1]);
        by += (double)elt * (x->r[k] * x->n[k] * x->r[k + 1] + y->r[k] * y->n[k] * y->r[k + 1]);
      }
    }
    const int pr = prof_begin(c, PK_DOT, fl, by);
    hipError_t e = launch_dot(dtype, dt, (int)tasks.size(), c->stream);
    prof_end(c, pr);
    if (e != hipSuccess) return hip_fail(c, e, "dot");
    c->ws_off -= bytes;   // chunk scratch is reused by the next chunk (stream ordered)
    c->ws_off = mark.off > c->ws_off ? mark.off : c->ws_off;
    i0 = i1;
  }
  const int32_t* dseg = upload(c, seg);
  const int32_t* didx = out_idx ? upload(c, *out_idx) : nullptr;
  if ((!seg.empty() && !dseg) || (out_idx && !out_idx->empty() && !didx)) return fail(c, TT_ENOMEM, "dot reduce tasks");
  hipError_t e = launch_segsum(slots, dseg, didx, npairs, out_dev, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "dot reduce");
  return TT_OK;
}

tt_status dot_pairs(tt_ctx* c, int npairs, const tt_sum* xs, const tt_sum* ys, double* out_dev) {
  return dot_pairs_idx(c, npairs, xs, ys, out_dev, nullptr);
}

}  // namespace tto

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* tt_status_str(tt_status s) {
  switch (s) {
    case TT_OK: return "ok";
    case TT_EINVAL: return "invalid argument";
    case TT_ENOMEM: return "out of memory (internal buffers)";
    case TT_ECAPACITY: return "workspace or output capacity too small";
    case TT_ENOTSPD: return "Gram matrix not positive definite";
    case TT_EBREAKDOWN: return "breakdown: zero vector after projection";
    case TT_ENONFINITE: return "non-finite value";
    case TT_EDEVICE: return "HIP runtime error";
    case TT_EGUARD: return "rank guard exceeded";
    case TT_ENOTIMPL: return "shape not supported";
  }
  return "unknown status";
}

tt_status tt_ctx_create(tt_ctx** ctx, int device, void* stream) {
  if (!ctx) return TT_EINVAL;
  *ctx = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TT_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return TT_EDEVICE;
  static bool lds_ready = false;  // LDS limits are per kernel, raised once per process
  if (!lds_ready) {
    if (qr_kernels_init() != hipSuccess) return TT_EDEVICE;
    lds_ready = true;
  }
  tt_ctx* c = new tt_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->pin.pinned = true;
  c->dev.pinned = false;
  *ctx = c;
  return TT_OK;
}

void tt_ctx_destroy(tt_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  prof_collect(c);
  for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->async_done) (void)hipEventDestroy(c->async_done);
  for (GraphEntry* g : c->graph_cache) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    g->arena.release();
    delete g;
  }
  c->graph_cache.clear();
  c->dev.release();
  c->pin.release();
  delete c;
}

tt_status tt_ctx_set_workspace(tt_ctx* c, void* ws, size_t bytes) {
  if (!c) return TT_EINVAL;
  if (ws && ((uintptr_t)ws & 255)) return fail(c, TT_EINVAL, "workspace must be 256-byte aligned");
  (void)hipSetDevice(c->device);
  wait_async(c);   // an asynchronous rounding may still use the old workspace
  c->ws = (char*)ws;
  c->ws_bytes = ws ? bytes : 0;
  c->ws_off = 0;
  return TT_OK;
}

size_t tt_ctx_required_bytes(const tt_ctx* c) { return c ? c->required : 0; }

const char* tt_last_error(const tt_ctx* c) { return c ? c->err.c_str() : "null context"; }

tt_status tt_ctx_set_autotune(tt_ctx* c, int on) {
  if (!c) return TT_EINVAL;
  c->autotune = on != 0;
  return TT_OK;
}

tt_status tt_tune_tsqr(tt_ctx* c, int64_t rows, int64_t cols, int32_t dtype, int32_t* leaf_rows, int32_t* fanin) {
  if (!c || rows < 1 || cols < 1 || (dtype != TT_F64 && dtype != TT_F32)) return fail(c, TT_EINVAL, "tune: bad shape");
  CallScope scope(c);
  const size_t mark = c->ws_off;
  c->ws_overflow = false;
  TreeShape best;
  tt_status s = tune_tree(c, rows, cols, dtype, &best);
  c->ws_off = mark;
  if (s != TT_OK) return s;
  if (!tuned_shape(rows, cols, dtype, nullptr)) {
    c->required = std::max(c->required, (size_t)(rows * cols * (int64_t)elt_size(dtype)) * 3 + (1 << 20));
    return fail(c, TT_ECAPACITY, "tune: workspace too small for the synthetic matrix and its tree");
  }
  if (leaf_rows) *leaf_rows = best.leaf_rows;
  if (fanin) *fanin = best.fanin;
  return TT_OK;
}

tt_status tt_ctx_set_profiling(tt_ctx* c, int on) {
  if (!c) return TT_EINVAL;
  c->prof = on != 0;
  for (int k = 0; k < PK_COUNT; ++k) {
    c->prof_ms[k] = c->prof_flops[k] = c->prof_bytes[k] = 0.0;
    c->prof_cnt[k] = 0;
  }
  return TT_OK;
}

tt_status tt_ctx_profile(const tt_ctx* c, int kind, double* ms, int64_t* launches, double* flops, double* bytes) {
  if (!c || kind < 0 || kind >= PK_COUNT) return TT_EINVAL;
  if (ms) *ms = c->prof_ms[kind];
  if (launches) *launches = c->prof_cnt[kind];
  if (flops) *flops = c->prof_flops[kind];
  if (bytes) *bytes = c->prof_bytes[kind];
  return TT_OK;
}

const char* tt_profile_kind_name(int kind) {
  static const char* names[PK_COUNT] = {"qr_factor_leaf", "qr_factor_node", "qr_apply", "svd_jacobi",
                                        "contraction_gemm", "tt_dot", "other"};
  return (kind >= 0 && kind < PK_COUNT) ? names[kind] : "unknown";
}

tt_status tt_dot_batched(tt_ctx* c, int32_t npairs, const tt_sum* xs, const tt_sum* ys, double* out) {
  if (!c || npairs < 0 || (npairs > 0 && (!xs || !ys || !out))) return fail(c, TT_EINVAL, "dot: bad arguments");
  if (npairs == 0) return TT_OK;
  CallScope scope(c);
  tt_status s;
  for (int p = 0; p < npairs; ++p) {
    if ((s = check_sum(c, &xs[p], "x")) != TT_OK) return s;
    if ((s = check_sum(c, &ys[p], "y")) != TT_OK) return s;
    if (!same_shape(xs[p].comp[0], ys[p].comp[0])) return fail(c, TT_EINVAL, "dot: shapes differ");
    if (xs[p].comp[0].dtype != xs[0].comp[0].dtype) return fail(c, TT_EINVAL, "dot: mixed dtypes in a batch");
  }
  double* dout = (double*)dev_scratch(c, (size_t)npairs * 8);
  double* hout = (double*)c->pin.alloc((size_t)npairs * 8);
  if (!dout || !hout) return fail(c, TT_ENOMEM, "dot output");
  if ((s = dot_pairs(c, npairs, xs, ys, dout)) != TT_OK) return s;
  hipError_t e = hipMemcpyAsync(hout, dout, (size_t)npairs * 8, hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "dot readback");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "dot sync");
  std::memcpy(out, hout, (size_t)npairs * 8);
  return TT_OK;
}

tt_status tt_dot(tt_ctx* c, const tt_sum* x, const tt_sum* y, double* out) {
  return tt_dot_batched(c, 1, x, y, out);
}

tt_status tt_axpy(tt_ctx* c, double alpha, const tt_vec* x, const tt_vec* y, tt_vec* z) {
  if (!c) return TT_EINVAL;
  tt_status s;
  if ((s = check_vec(c, x, "x", true)) != TT_OK) return s;
  if ((s = check_vec(c, y, "y", true)) != TT_OK) return s;
  if ((s = check_vec(c, z, "z", false)) != TT_OK) return s;
  if (!same_shape(*x, *y) || !same_shape(*x, *z)) return fail(c, TT_EINVAL, "axpy: operands differ in d, n or dtype");
  if (!std::isfinite(alpha)) return fail(c, TT_EINVAL, "axpy: non-finite alpha");
  const int d = x->d;
  int64_t zr[TT_MAXD + 1];
  zr[0] = zr[d] = 1;
  for (int k = 1; k < d; ++k) zr[k] = x->r[k] + y->r[k];
  int64_t need = 0;
  for (int k = 0; k < d; ++k) need += zr[k] * x->n[k] * zr[k + 1];
  if (z->capacity < need) return fail(c, TT_ECAPACITY, "axpy: z capacity " + std::to_string(z->capacity) +
                                                           " < " + std::to_string(need));
  CallScope scope(c);
  const size_t elt = elt_size(x->dtype);
  std::vector<AxpyTask> tasks;
  int64_t xo = 0, yo = 0, zo = 0, maxe = 0;
  for (int k = 0; k < d; ++k) {
    AxpyTask t;
    std::memset(&t, 0, sizeof(t));
    t.x = (const char*)x->data + (size_t)xo * elt;
    t.y = (const char*)y->data + (size_t)yo * elt;
    t.z = (char*)z->data + (size_t)zo * elt;
    t.n = (int32_t)x->n[k];
    t.xr0 = (int32_t)x->r[k];
    t.xr1 = (int32_t)x->r[k + 1];
    t.yr0 = (int32_t)y->r[k];
    t.yr1 = (int32_t)y->r[k + 1];
    t.first = (k == 0);
    t.last = (k == d - 1);
    t.alpha = (k == 0) ? alpha : 1.0;
    tasks.push_back(t);
    xo += x->r[k] * x->n[k] * x->r[k + 1];
    yo += y->r[k] * y->n[k] * y->r[k + 1];
    const int64_t ze = zr[k] * x->n[k] * zr[k + 1];
    zo += ze;
    maxe = std::max(maxe, ze);
  }
  const AxpyTask* dt = upload(c, tasks);
  if (!dt) return fail(c, TT_ENOMEM, "axpy tasks");
  hipError_t e = launch_axpy(x->dtype, dt, (int)tasks.size(), maxe, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "axpy");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "axpy sync");
  for (int k = 0; k <= d; ++k) z->r[k] = zr[k];
  return TT_OK;
}

int64_t tt_round_out_capacity(const tt_sum* x) {
  if (!x || x->ncomp < 1 || !x->comp) return -1;
  const tt_vec& v = x->comp[0];
  if (v.d < 1 || v.d > TT_MAXD) return -1;
  int64_t caps[TT_MAXD + 1], R[TT_MAXD + 1];
  rank_caps(v, caps);
  for (int k = 0; k <= v.d; ++k) {
    R[k] = 0;
    for (int i = 0; i < x->ncomp; ++i) R[k] += x->comp[i].r[k];
  }
  R[0] = R[v.d] = 1;
  int64_t s = 0;
  for (int k = 0; k < v.d; ++k) s += std::min(R[k], caps[k]) * v.n[k] * std::min(R[k + 1], caps[k + 1]);
  return s;
}

double tt_round_effective_delta(const tt_sum* x, double delta) {
  if (!x || x->ncomp < 1 || !x->comp || !(delta >= 0.0)) return -1.0;
  const tt_vec& s0 = x->comp[0];
  if (s0.d < 1 || s0.d > TT_MAXD) return -1.0;
  if (s0.dtype != TT_F32 || s0.d == 1) return delta;
  int64_t caps[TT_MAXD + 1];
  rank_caps(s0, caps);
  int64_t smax = 1;
  for (int k = 1; k < s0.d; ++k) {
    int64_t R = 0;
    for (int c = 0; c < x->ncomp; ++c) R += x->comp[c].r[k];
    smax = std::max(smax, std::min(R, caps[k]));
  }
  return std::max(delta, std::sqrt((double)(s0.d - 1)) * fp32_eps_floor(smax));
}

int64_t tt_round_workspace_bytes(const tt_sum* x) {
  if (!x || x->ncomp < 1 || !x->comp) return -1;
  std::vector<RJob> jobs(1);
  make_job(nullptr, x, 0.0, 0, nullptr, jobs[0]);
  return round_workspace_bytes(jobs);
}

tt_status tt_round_batched(tt_ctx* c, int32_t njobs, const tt_sum* xs, const double* deltas,
                           const int64_t* max_ranks, tt_vec* outs, tt_status* job_status) {
  if (!c || njobs < 0 || (njobs > 0 && (!xs || !deltas || !outs))) return fail(c, TT_EINVAL, "round: bad arguments");
  if (njobs == 0) return TT_OK;
  tt_status s;
  for (int j = 0; j < njobs; ++j) {
    if ((s = check_sum(c, &xs[j], "x")) != TT_OK) return s;
    if ((s = check_vec(c, &outs[j], "out", false)) != TT_OK) return s;
    if (!same_shape(xs[j].comp[0], outs[j])) return fail(c, TT_EINVAL, "round: out shape differs from x");
    if (!(deltas[j] >= 0.0) || !std::isfinite(deltas[j])) return fail(c, TT_EINVAL, "round: delta must be >= 0");
    if (xs[j].comp[0].dtype != xs[0].comp[0].dtype) return fail(c, TT_EINVAL, "round: mixed dtypes in a batch");
  }
  CallScope scope(c);
  std::vector<RJob> jobs(njobs);
  for (int j = 0; j < njobs; ++j)
    make_job(c, &xs[j], deltas[j], max_ranks ? max_ranks[j] : 0, &outs[j], jobs[j]);
  s = round_jobs(c, jobs);
  if (s != TT_OK) return s;
  tt_status first = TT_OK;
  for (int j = 0; j < njobs; ++j) {
    if (job_status) job_status[j] = jobs[j].status;
    if (first == TT_OK && jobs[j].status != TT_OK) first = jobs[j].status;
  }
  if (first != TT_OK && c->err.empty()) c->err = "one or more jobs failed (see job_status)";
  return first;
}

tt_status tt_round_batched_async(tt_ctx* c, int32_t njobs, const tt_sum* xs, const double* deltas,
                                 const int64_t* max_ranks, tt_vec* outs, int32_t* ranks, int32_t* job_status,
                                 double* norms) {
  if (!c || njobs < 0 || (njobs > 0 && (!xs || !deltas || !outs || !ranks || !job_status)))
    return fail(c, TT_EINVAL, "round async: bad arguments");
  if (njobs == 0) return TT_OK;
  if (c->prof) return fail(c, TT_EINVAL, "round async: the per-launch profiler needs the synchronous calls");
  tt_status s;
  for (int j = 0; j < njobs; ++j) {
    if ((s = check_sum(c, &xs[j], "x")) != TT_OK) return s;
    if ((s = check_vec(c, &outs[j], "out", false)) != TT_OK) return s;
    if (!same_shape(xs[j].comp[0], outs[j])) return fail(c, TT_EINVAL, "round: out shape differs from x");
    if (!(deltas[j] >= 0.0) || !std::isfinite(deltas[j])) return fail(c, TT_EINVAL, "round: delta must be >= 0");
    if (xs[j].comp[0].dtype != xs[0].comp[0].dtype) return fail(c, TT_EINVAL, "round: mixed dtypes in a batch");
  }
  CallScope scope(c);
  if (!c->async_done && hipEventCreateWithFlags(&c->async_done, hipEventDisableTiming) != hipSuccess)
    return fail(c, TT_EDEVICE, "event");
  RoundMode mode;
  mode.bound_plan = true;
  mode.async = true;
  mode.ranks = ranks;
  mode.status = job_status;
  mode.norms = norms;
  auto run = [&]() -> tt_status {
    std::vector<RJob> jobs(njobs);
    for (int j = 0; j < njobs; ++j)
      make_job(c, &xs[j], deltas[j], max_ranks ? max_ranks[j] : 0, &outs[j], jobs[j]);
    return round_jobs(c, jobs, mode);
  };
  if (!c->graphs) {
    s = run();
    if (s != TT_OK) return s;
    scope.async = true;
    return TT_OK;
  }
  // graph replay: the exact bytes of every argument that reaches a launch (pointers, shapes,
  // coefficients, accuracies, capacities, workspace) name the entry
  std::string sig;
  auto put = [&](const void* p, size_t n) { sig.append((const char*)p, n); };
  put(&njobs, sizeof(njobs));
  put(&c->ws, sizeof(c->ws));
  put(&c->ws_bytes, sizeof(c->ws_bytes));
  put(&c->stream, sizeof(c->stream));
  put(&ranks, sizeof(ranks));
  put(&job_status, sizeof(job_status));
  put(&norms, sizeof(norms));
  for (int j = 0; j < njobs; ++j) {
    put(&xs[j].ncomp, sizeof(int32_t));
    for (int i = 0; i < xs[j].ncomp; ++i) {
      const tt_vec& v = xs[j].comp[i];
      put(&xs[j].coef[i], sizeof(double));
      put(&v.d, sizeof(v.d));
      put(&v.dtype, sizeof(v.dtype));
      put(v.n, sizeof(int64_t) * v.d);
      put(v.r, sizeof(int64_t) * (v.d + 1));
      put(&v.data, sizeof(v.data));
    }
    put(&deltas[j], sizeof(double));
    const int64_t mr = max_ranks ? max_ranks[j] : 0;
    put(&mr, sizeof(mr));
    put(&outs[j].data, sizeof(outs[j].data));
    put(&outs[j].capacity, sizeof(outs[j].capacity));
  }
  GraphEntry* ent = nullptr;
  for (GraphEntry* g : c->graph_cache)
    if (g->sig == sig) ent = g;
  ++c->graph_clock;
  if (ent && ent->exec) {
    ent->last_use = c->graph_clock;
    hipError_t e = hipGraphLaunch(ent->exec, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "graph launch");
    scope.async = true;
    return TT_OK;
  }
  if (ent) {   // not capturable: run directly
    s = run();
    if (s != TT_OK) return s;
    scope.async = true;
    return TT_OK;
  }
  if (c->graph_cache.size() >= 16) {   // drop the least recently used entry
    auto it = std::min_element(c->graph_cache.begin(), c->graph_cache.end(),
                               [](const GraphEntry* a, const GraphEntry* b) { return a->last_use < b->last_use; });
    (void)hipStreamSynchronize(c->stream);
    if ((*it)->exec) (void)hipGraphExecDestroy((*it)->exec);
    (*it)->arena.release();
    delete *it;
    c->graph_cache.erase(it);
  }
  ent = new GraphEntry;
  ent->sig = sig;
  ent->last_use = c->graph_clock;
  c->graph_cache.push_back(ent);
  // pass 1: run the call, its descriptors going to the entry's block (again when it tuned
  // tree shapes on the way: the tuning's own allocations must not shift the block's layout)
  c->graph_arena = &ent->arena;
  for (int pass = 0; pass < 2; ++pass) {
    const uint64_t tuned = c->tune_count;
    ent->arena.rewind();
    s = run();
    if (s != TT_OK) {
      c->graph_arena = nullptr;
      return s;
    }
    if (c->tune_count == tuned) break;
  }
  // pass 2: capture the same launches (the block already holds their descriptors)
  ent->arena.rewind();
  c->graph_capturing = true;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  tt_status cs = TT_OK;
  if (e == hipSuccess) {
    const std::string keep_err = c->err;
    cs = run();
    hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
    if (cs == TT_OK && e2 == hipSuccess && graph) {
      if (hipGraphInstantiate(&ent->exec, graph, nullptr, nullptr, 0) != hipSuccess) ent->exec = nullptr;
    }
    if (graph) (void)hipGraphDestroy(graph);
    c->err = keep_err;
  }
  (void)hipGetLastError();   // a failed capture leaves the entry without a graph: later calls run directly
  c->graph_capturing = false;
  c->graph_arena = nullptr;
  scope.async = true;
  return TT_OK;
}

tt_status tt_ctx_set_svd_block_min(tt_ctx* c, int32_t rows) {
  if (!c) return TT_EINVAL;
  if (rows < 32 || rows > SVD_SMALL_MAX) return fail(c, TT_EINVAL, "svd block crossover must be in [32, 1024]");
  c->svd_block_min = rows;
  return TT_OK;
}

tt_status tt_ctx_set_graphs(tt_ctx* c, int on) {
  if (!c) return TT_EINVAL;
  (void)hipSetDevice(c->device);
  wait_async(c);
  if (!on) {
    (void)hipStreamSynchronize(c->stream);
    for (GraphEntry* g : c->graph_cache) {
      if (g->exec) (void)hipGraphExecDestroy(g->exec);
      g->arena.release();
      delete g;
    }
    c->graph_cache.clear();
  }
  c->graphs = on != 0;
  return TT_OK;
}

int32_t tt_ctx_graph_count(const tt_ctx* c) {
  if (!c) return -1;
  int32_t n = 0;
  for (const GraphEntry* g : c->graph_cache) n += g->exec ? 1 : 0;
  return n;
}

tt_status tt_norm(tt_ctx* c, const tt_sum* x, double* out) {
  if (!c) return TT_EINVAL;
  tt_status s;
  if ((s = check_sum(c, x, "x")) != TT_OK) return s;
  if (!out) return fail(c, TT_EINVAL, "norm: out is NULL");
  CallScope scope(c);
  std::vector<RJob> jobs(1);
  make_job(c, x, 0.0, 0, nullptr, jobs[0]);
  jobs[0].orth_only = true;
  s = round_jobs(c, jobs);
  if (s != TT_OK) return s;
  if (jobs[0].status != TT_OK) return fail(c, jobs[0].status, "norm failed");
  *out = jobs[0].norm;
  return TT_OK;
}

tt_status tt_round(tt_ctx* c, const tt_sum* x, double delta, int64_t max_rank, tt_vec* out, double* norm_x) {
  if (!c) return TT_EINVAL;
  tt_status s;
  if ((s = check_sum(c, x, "x")) != TT_OK) return s;
  if ((s = check_vec(c, out, "out", false)) != TT_OK) return s;
  if (!same_shape(x->comp[0], *out)) return fail(c, TT_EINVAL, "round: out shape differs from x");
  if (!(delta >= 0.0) || !std::isfinite(delta)) return fail(c, TT_EINVAL, "round: delta must be >= 0");
  CallScope scope(c);
  std::vector<RJob> jobs(1);
  make_job(c, x, delta, max_rank, out, jobs[0]);
  s = round_jobs(c, jobs);
  if (s != TT_OK) return s;
  if (jobs[0].status != TT_OK) return fail(c, jobs[0].status, "round: output capacity too small");
  if (norm_x) *norm_x = jobs[0].norm;
  return TT_OK;
}

// ----------------------------------------------------------------------------
// Orthogonalization schemes (Section 3, Algorithms 1-5)
// ----------------------------------------------------------------------------
namespace {

int64_t max_bond(const int64_t* R, int d) {
  int64_t m = 0;
  for (int k = 1; k < d; ++k) m = std::max(m, R[k]);
  return m;
}

tt_status read_doubles(tt_ctx* c, const double* dsrc, double* hdst, size_t n) {
  if (n == 0) return TT_OK;
  double* h = (double*)c->pin.alloc(n * 8);
  if (!h) return fail(c, TT_ENOMEM, "readback");
  hipError_t e = hipMemcpyAsync(h, dsrc, n * 8, hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "readback");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "sync");
  std::memcpy(hdst, h, n * 8);
  return TT_OK;
}

tt_status round_one(tt_ctx* c, const tt_sum* x, double delta, tt_vec* out) {
  std::vector<RJob> jobs(1);
  make_job(c, x, delta, 0, out, jobs[0]);
  tt_status s = round_jobs(c, jobs);
  if (s != TT_OK) return s;
  if (jobs[0].status != TT_OK) return fail(c, jobs[0].status, "rounding output capacity too small");
  return TT_OK;
}

// Gq[i][j] = <q_i, q_j> for j <= i, then mirror into the upper triangle.
tt_status gram_row(tt_ctx* c, int i, int m, const tt_vec* q, double* Gq) {
  std::vector<tt_sum> xs(i + 1), ys(i + 1);
  static const double one = 1.0;
  for (int j = 0; j <= i; ++j) {
    xs[j] = tt_sum{1, &one, &q[i]};
    ys[j] = tt_sum{1, &one, &q[j]};
  }
  tt_status s = dot_pairs(c, i + 1, xs.data(), ys.data(), Gq + (size_t)i * m);
  if (s != TT_OK) return s;
  hipError_t e = launch_sym_lower(Gq, m, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "sym");
  return TT_OK;
}

// Singular values of the leading blocks of the FP64 Gram matrix Gq (m x m):
// of I - G_k when minus_identity (its largest is ||I_k - Q_k^T Q_k||_2, Section
// 3.4), else of G_k itself.  sig_host[k-1] receives the k values of block k
// (sorted decreasing) at offset (k-1)k/2.
tt_status block_spectra(tt_ctx* c, const double* Gq, int m, int minus_identity, double* sig_host) {
  size_t esz = 0;
  for (int k = 1; k <= m; ++k) esz += (size_t)k * k;
  double* E = (double*)dev_scratch(c, esz * 8);
  double* scratch = (double*)dev_scratch(c, (size_t)m * (4 * (size_t)m * m + 4 * m) * 8);
  double* zero = (double*)dev_scratch(c, 8);
  int32_t* ranks = (int32_t*)dev_scratch(c, (size_t)m * 4);
  if (!E || !scratch || !zero || !ranks) return fail(c, TT_ENOMEM, "loo buffers");
  hipError_t e = hipMemsetAsync(zero, 0, 8, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "loo");
  if ((e = launch_loo_mats(Gq, m, E, minus_identity, c->stream)) != hipSuccess) return hip_fail(c, e, "loo mats");
  std::vector<SvdTask> tasks;
  size_t eo = 0, so = 0;
  for (int k = 1; k <= m; ++k) {
    SvdTask t;
    std::memset(&t, 0, sizeof(t));
    t.R = E + eo;
    t.r_ld = k;
    t.kr = k;
    t.ncol = k;
    t.upper = 0;
    t.A = scratch + so;
    so += (size_t)k * k;
    t.acc = scratch + so;
    so += (size_t)k * k;
    t.sigma = scratch + so;
    so += k;
    t.perm = (int32_t*)(scratch + so);
    so += k;
    t.norm = zero;
    t.delta_scaled = 0.0;
    t.max_rank = 0;
    t.rank_out = ranks + (k - 1);
    t.wt = scratch + so;
    so += (size_t)k * k;
    t.ur = scratch + so;
    so += (size_t)k * k;
    tasks.push_back(t);
    eo += (size_t)k * k;
  }
  const SvdTask* dt = upload(c, tasks);
  if (!dt) return fail(c, TT_ENOMEM, "loo tasks");
  if ((e = launch_svd(dt, m, c->stream)) != hipSuccess) return hip_fail(c, e, "loo svd");
  for (int k = 1; k <= m; ++k) {
    tt_status s = read_doubles(c, tasks[k - 1].sigma, sig_host + (size_t)(k - 1) * k / 2, k);
    if (s != TT_OK) return s;
  }
  return TT_OK;
}

tt_status loo_from_gram(tt_ctx* c, const double* Gq, int m, double* loo_host) {
  std::vector<double> sig((size_t)m * (m + 1) / 2);
  tt_status s = block_spectra(c, Gq, m, 1, sig.data());
  if (s != TT_OK) return s;
  for (int k = 1; k <= m; ++k) loo_host[k - 1] = sig[(size_t)(k - 1) * k / 2];
  return TT_OK;
}

// A lazy sum under construction: coefficients and components on the host.
struct LazySum {
  std::vector<double> coef;
  std::vector<tt_vec> comp;
  void add(double a, const tt_vec& v) {
    coef.push_back(a);
    comp.push_back(v);
  }
  tt_sum view() const { return tt_sum{(int32_t)comp.size(), coef.data(), comp.data()}; }
};

// Packed size of a TT of shape `shape` whose bond ranks are b (already capped).
int64_t packed_size(const tt_vec& shape, const int64_t* b) {
  int64_t s = 0;
  for (int k = 0; k < shape.d; ++k) s += b[k] * shape.n[k] * b[k + 1];
  return s;
}

// TT-Householder (Section 3.3, Algorithms 6-8).  For i = 0..m-1: the Householder
// TT-vector u_i of the (rounded) running vector w against e_0..e_i (two
// roundings), column i of R, the reflection of the later a~_j by u_i (a term
// appended to their lazy sums), and w = round(a~_{i+1}).  Then q_i = H_0..H_i e_i
// and the m final roundings in one batch.  Every a~_j and q~_i is a lazy sum of
// one original vector and Householder vectors, so each inner product with u_i is
// taken in component form: the original's product with u_i plus the earlier
// coefficients times the Gram matrix of the u (the same sum, each <u_l, u_i>
// computed once instead of once per vector).  The reflection of a~_i by its own
// u_i is skipped: the algorithm never reads that result.  The u_i, two slots for w and one for the
// first rounding of each u live in the workspace at sizes bounded before any
// work starts (bond ranks of a rounded sum are at most those of the sum and the
// rank caps).
tt_status ortho_householder(tt_ctx* c, int m, const tt_sum* a, double delta, int64_t rank_guard, tt_vec* q,
                            double* Rdev, double* R, double* loo, double* Gq, tt_ortho_stats& st) {
  const tt_vec& s0 = a[0].comp[0];
  const int d = s0.d;
  const size_t esz = elt_size(s0.dtype);
  hipError_t e;
  tt_status s;
  {
    // the canonical basis must have m elements
    int64_t total = 1;
    for (int k = 0; k < d && total < m; ++k) total = std::min<int64_t>(total * s0.n[k], (int64_t)m);
    if (total < m) return fail(c, TT_EINVAL, "householder: m exceeds the number of tensor entries");
  }
  int64_t caps[TT_MAXD + 1];
  rank_caps(s0, caps);
  auto cap_of = [&](int64_t* b) {
    for (int k = 0; k <= d; ++k) {
      b[k] = std::min(b[k], caps[k]);
      if (rank_guard > 0) b[k] = std::min(b[k], rank_guard);
    }
    b[0] = b[d] = 1;
  };
  // a-priori bond bounds: w_0 = a_0; w_i <= a_i + sum_{l<i} u_l; first rounding <= w_i + i; u_i <= that + 1
  std::vector<int64_t> bu((size_t)m * (d + 1)), sumu(d + 1, 0);
  int64_t wmax = 0, w1max = 0;
  std::vector<int64_t> uoff(m + 1, 0);
  for (int i = 0; i < m; ++i) {
    int64_t bw[TT_MAXD + 1], b1[TT_MAXD + 1];
    for (int k = 0; k <= d; ++k) {
      int64_t ra = 0;
      for (int cc = 0; cc < a[i].ncomp; ++cc) ra += a[i].comp[cc].r[k];
      bw[k] = ra + sumu[k];
    }
    cap_of(bw);
    for (int k = 0; k <= d; ++k) b1[k] = bw[k] + i;
    cap_of(b1);
    int64_t* u = &bu[(size_t)i * (d + 1)];
    for (int k = 0; k <= d; ++k) u[k] = b1[k] + 1;
    cap_of(u);
    for (int k = 0; k <= d; ++k) sumu[k] += u[k];
    if (i > 0) wmax = std::max(wmax, packed_size(s0, bw));
    w1max = std::max(w1max, packed_size(s0, b1));
    uoff[i + 1] = uoff[i] + ((packed_size(s0, u) * (int64_t)esz + 255) & ~(int64_t)255) / (int64_t)esz;
  }
  int64_t S = 0;
  for (int k = 0; k < d; ++k) S += s0.n[k];
  char* Ebuf = (char*)ws_alloc(c, (size_t)m * S * esz);
  char* Ubuf = (char*)ws_alloc(c, (size_t)uoff[m] * esz);
  char* Wbuf[2] = {(char*)ws_alloc(c, (size_t)std::max<int64_t>(wmax, 1) * esz),
                   (char*)ws_alloc(c, (size_t)std::max<int64_t>(wmax, 1) * esz)};
  char* W1buf = (char*)ws_alloc(c, (size_t)w1max * esz);
  if (!Ebuf || !Ubuf || !Wbuf[0] || !Wbuf[1] || !W1buf)
    return fail(c, TT_ECAPACITY, "workspace too small for the Householder vectors: need " + std::to_string(c->required));
  const size_t top = c->ws_off;
  const int64_t* dn = (const int64_t*)upload_bytes(c, s0.n, (size_t)d * 8);
  double* dots = (double*)dev_scratch(c, (size_t)(m + 1) * 8);
  double* coefd = (double*)dev_scratch(c, (size_t)(m + 1) * 8);
  double* nrm = (double*)dev_scratch(c, 8);
  // hbuf: <a_j, u_i> (first m) and the Gram matrix of the u (Gu = hbuf + m, row i holds
  // <u_l, u_i>, l < i); Ct[l*m + j] = reflection coefficient of a~_j by u_l; EU[i*m + j] =
  // <e_i, u_j>; Dq[i*m + j] = coefficient of u_j in q_i
  double* hbuf = (double*)dev_scratch(c, (size_t)(m + m * m) * 8);
  double* Ct = (double*)dev_scratch(c, (size_t)m * m * 8);
  double* EU = (double*)dev_scratch(c, (size_t)m * m * 8);
  double* Dq = (double*)dev_scratch(c, (size_t)m * m * 8);
  if (!dn || !dots || !coefd || !nrm || !hbuf || !Ct || !EU || !Dq) return fail(c, TT_ENOMEM, "householder buffers");
  double* Gu = hbuf + m;
  if ((e = launch_canonical(s0.dtype, Ebuf, dn, d, S, 0, m, c->stream)) != hipSuccess)
    return hip_fail(c, e, "canonical basis");
  auto make_vec = [&](void* data, int64_t capacity) {
    tt_vec v = s0;
    for (int k = 0; k <= d; ++k) v.r[k] = 1;
    v.data = data;
    v.capacity = capacity;
    return v;
  };
  std::vector<tt_vec> E(m), U(m);
  for (int i = 0; i < m; ++i) E[i] = make_vec(Ebuf + (size_t)i * S * esz, S);
  static const double one = 1.0;
  std::vector<LazySum> At(m);   // a~_j
  for (int j = 0; j < m; ++j)
    for (int cc = 0; cc < a[j].ncomp; ++cc) At[j].add(a[j].coef[cc], a[j].comp[cc]);

  // one rounding of `sum` into `out`, with the rank guard and the statistics
  auto round_into = [&](const tt_sum& sum, tt_vec* out) -> tt_status {
    RJob probe;
    make_job(c, &sum, delta, 0, nullptr, probe);
    const int64_t pre = max_bond(probe.R, d);
    st.max_pre_rank = (int32_t)std::max<int64_t>(st.max_pre_rank, pre);
    if (rank_guard > 0 && pre > rank_guard)
      return fail(c, TT_EGUARD, "pre-round rank " + std::to_string(pre) + " exceeds the guard");
    tt_status rs = round_one(c, &sum, delta, out);
    if (rs != TT_OK) return rs;
    ++st.rounds;
    st.max_post_rank = (int32_t)std::max<int64_t>(st.max_post_rank, max_bond(out->r, d));
    return TT_OK;
  };

  tt_vec w;                 // the running vector fed to the next Householder TT-vector
  tt_sum wsum = a[0];       // w_0 = a_0 as given
  std::vector<double> hc(m + 1);
  for (int i = 0; i < m; ++i) {
    c->ws_off = top;
    // dots <w, e_j> (j <= i) and ||w||^2, then column i of R.  A rounded w has
    // left-orthonormal cores 0..d-2, so its norm is that of its last core; w_0 = a_0
    // is a lazy sum and takes <w, w>.
    {
      const int np = (i == 0) ? i + 2 : i + 1;
      std::vector<tt_sum> xs(np, wsum), ys(np, wsum);
      for (int j = 0; j <= i; ++j) ys[j] = tt_sum{1, &one, &E[j]};
      if ((s = dot_pairs(c, np, xs.data(), ys.data(), dots)) != TT_OK) return s;
      if (i > 0) {
        int64_t off = 0;
        for (int k = 0; k + 1 < d; ++k) off += w.r[k] * w.n[k] * w.r[k + 1];
        if ((e = launch_sumsq(w.dtype, (const char*)w.data + (size_t)off * esz, w.r[d - 1] * w.n[d - 1], dots + i + 1,
                              c->stream)) != hipSuccess)
          return hip_fail(c, e, "norm of w");
      }
    }
    if ((e = launch_hh_column(dots, i, i > 0 ? 1 : 0, Rdev + (size_t)i * m, coefd, c->stream)) != hipSuccess)
      return hip_fail(c, e, "householder column");
    if ((s = read_doubles(c, coefd, hc.data(), i + 1)) != TT_OK) return s;
    if (!(hc[i] != 0.0) || !std::isfinite(hc[i]))
      return fail(c, TT_EBREAKDOWN, "householder: vector " + std::to_string(i) + " lies in the span of the earlier ones");
    // first rounding: w - sum_{j<i} R(j, i) e_j
    LazySum p1;
    for (int cc = 0; cc < wsum.ncomp; ++cc) p1.add(wsum.coef[cc], wsum.comp[cc]);
    for (int j = 0; j < i; ++j) p1.add(hc[j], E[j]);
    tt_vec w1 = make_vec(W1buf, w1max);
    if ((s = round_into(p1.view(), &w1)) != TT_OK) return s;
    // second rounding: w1 - R(i, i) e_i, normalised
    U[i] = make_vec(Ubuf + (size_t)uoff[i] * esz, uoff[i + 1] - uoff[i]);
    LazySum p2;
    p2.add(1.0, w1);
    p2.add(hc[i], E[i]);
    if ((s = round_into(p2.view(), &U[i])) != TT_OK) return s;
    int64_t off = 0;
    for (int k = 0; k + 1 < d; ++k) off += U[i].r[k] * U[i].n[k] * U[i].r[k + 1];
    const int64_t last = U[i].r[d - 1] * U[i].n[d - 1];
    char* lastp = (char*)U[i].data + (size_t)off * esz;
    if ((e = launch_sumsq(U[i].dtype, lastp, last, nrm, c->stream)) != hipSuccess) return hip_fail(c, e, "norm");
    double hn = 0.0;
    if ((s = read_doubles(c, nrm, &hn, 1)) != TT_OK) return s;
    if (!(hn > 0.0) || !std::isfinite(hn))
      return fail(c, TT_EBREAKDOWN, "householder: zero Householder vector at " + std::to_string(i));
    if ((e = launch_scale(U[i].dtype, lastp, last, nrm, c->stream)) != hipSuccess) return hip_fail(c, e, "scale");
    // reflect a~_j, j > i:  a~_j -= 2 <a~_j, u_i> u_i, the inner product in component
    // form from <a_j, u_i> and row i of the Gram matrix of the u (one batch)
    const int nr = m - 1 - i;
    {
      std::vector<tt_sum> xs, ys;
      std::vector<int32_t> idx;
      const tt_sum ui{1, &one, &U[i]};
      for (int j = i + 1; j < m; ++j) {
        xs.push_back(a[j]);
        ys.push_back(ui);
        idx.push_back(j - i - 1);
      }
      for (int l = 0; l < i; ++l) {
        xs.push_back(tt_sum{1, &one, &U[l]});
        ys.push_back(ui);
        idx.push_back(m + i * m + l);
      }
      if (!xs.empty() && (s = dot_pairs_idx(c, (int)xs.size(), xs.data(), ys.data(), hbuf, &idx)) != TT_OK) return s;
    }
    if (nr > 0) {
      if ((e = launch_hh_reflect(hbuf, Gu, Ct, m, i, c->stream)) != hipSuccess) return hip_fail(c, e, "reflect");
      if ((s = read_doubles(c, Ct + (size_t)i * m + i + 1, hc.data(), nr)) != TT_OK) return s;
      for (int j = 0; j < nr; ++j) At[i + 1 + j].add(hc[j], U[i]);
      // w = round(a~_{i+1})
      w = make_vec(Wbuf[(i + 1) & 1], wmax);
      if ((s = round_into(At[i + 1].view(), &w)) != TT_OK) return s;
      wsum = tt_sum{1, &one, &w};
    }
  }
  // q_i = H_0 ... H_i e_i: <e_i, u_j> for j <= i in one batch, then the
  // coefficients of every q_i from one recurrence kernel over the Gram matrix of the u
  c->ws_off = top;
  {
    std::vector<tt_sum> xs, ys;
    std::vector<int32_t> idx;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j <= i; ++j) {
        xs.push_back(tt_sum{1, &one, &E[i]});
        ys.push_back(tt_sum{1, &one, &U[j]});
        idx.push_back(i * m + j);
      }
    if ((s = dot_pairs_idx(c, (int)xs.size(), xs.data(), ys.data(), EU, &idx)) != TT_OK) return s;
  }
  if ((e = launch_hh_qcoef(EU, Gu, Dq, m, c->stream)) != hipSuccess) return hip_fail(c, e, "q coefficients");
  std::vector<double> hD((size_t)m * m);
  if ((s = read_doubles(c, Dq, hD.data(), hD.size())) != TT_OK) return s;
  std::vector<LazySum> Qs(m);
  for (int i = 0; i < m; ++i) {
    Qs[i].add(1.0, E[i]);
    for (int j = i; j >= 0; --j) Qs[i].add(hD[(size_t)i * m + j], U[j]);
  }
  std::vector<tt_sum> qsums(m);
  std::vector<RJob> jobs(m);
  for (int i = 0; i < m; ++i) {
    qsums[i] = Qs[i].view();
    make_job(c, &qsums[i], delta, 0, &q[i], jobs[i]);
    const int64_t pre = max_bond(jobs[i].R, d);
    st.max_pre_rank = (int32_t)std::max<int64_t>(st.max_pre_rank, pre);
    if (st.q_pre_size) st.q_pre_size[i] = packed_size(a[0].comp[0], jobs[i].R);
    if (rank_guard > 0 && pre > rank_guard)
      return fail(c, TT_EGUARD, "pre-round rank " + std::to_string(pre) + " of q exceeds the guard");
  }
  if ((s = round_jobs_grouped(c, jobs)) != TT_OK) return s;
  for (auto& jb : jobs) {
    if (jb.status != TT_OK) return fail(c, jb.status, "householder: output capacity of q");
    st.max_post_rank = (int32_t)std::max<int64_t>(st.max_post_rank, max_bond(jb.out->r, d));
  }
  st.rounds += m;
  st.m_reached = m;
  if ((s = read_doubles(c, Rdev, R, (size_t)m * m)) != TT_OK) return s;
  if (loo) {
    for (int i = 0; i < m; ++i)
      if ((s = gram_row(c, i, m, q, Gq)) != TT_OK) return s;
    if ((s = loo_from_gram(c, Gq, m, loo)) != TT_OK) return s;
  }
  return TT_OK;
}

}  // namespace

tt_status tt_round_randomized(tt_ctx* c, const tt_sum* x, const tt_vec* sketch, double delta, tt_vec* out) {
  if (!c) return TT_EINVAL;
  tt_status s;
  if ((s = check_sum(c, x, "x")) != TT_OK) return s;
  if ((s = check_vec(c, sketch, "sketch", true)) != TT_OK) return s;
  if ((s = check_vec(c, out, "out", false)) != TT_OK) return s;
  const tt_vec& s0 = x->comp[0];
  if (sketch->dtype != TT_F64) return fail(c, TT_EINVAL, "randomized rounding: the sketch must be FP64");
  bool shape_ok = sketch->d == s0.d;
  for (int k = 0; shape_ok && k < s0.d; ++k) shape_ok = sketch->n[k] == s0.n[k];
  if (!shape_ok || !same_shape(s0, *out))
    return fail(c, TT_EINVAL, "randomized rounding: x, sketch and out differ in d or n (or x and out in dtype)");
  if (!(delta >= 0.0) || !std::isfinite(delta)) return fail(c, TT_EINVAL, "randomized rounding: delta must be >= 0");
  for (int k = 1; k < s0.d; ++k)
    if (sketch->r[k] > 1024) return fail(c, TT_ENOTIMPL, "randomized rounding: sketch rank above 1024");
  CallScope scope(c);
  if (s0.d == 1) return round_one(c, x, delta, out);
  return round_randomized(c, x, sketch, delta, out);
}

tt_status tt_laplacian(tt_ctx* c, const tt_vec* x, double alpha, tt_vec* out) {
  if (!c) return TT_EINVAL;
  tt_status s;
  if ((s = check_vec(c, x, "x", true)) != TT_OK) return s;
  if ((s = check_vec(c, out, "out", false)) != TT_OK) return s;
  if (!same_shape(*x, *out)) return fail(c, TT_EINVAL, "laplacian: out differs from x in d, n or dtype");
  if (!std::isfinite(alpha)) return fail(c, TT_EINVAL, "laplacian: non-finite alpha");
  if (x->data == out->data) return fail(c, TT_EINVAL, "laplacian: out must not alias x");
  const int d = x->d;
  int64_t yr[TT_MAXD + 1];
  yr[0] = yr[d] = 1;
  for (int k = 1; k < d; ++k) yr[k] = 2 * x->r[k];
  int64_t need = 0;
  for (int k = 0; k < d; ++k) need += yr[k] * x->n[k] * yr[k + 1];
  if (out->capacity < need)
    return fail(c, TT_ECAPACITY, "laplacian: out capacity " + std::to_string(out->capacity) + " < " + std::to_string(need));
  CallScope scope(c);
  const size_t esz = elt_size(x->dtype);
  int64_t xo = 0, yo = 0;
  for (int k = 0; k < d; ++k) {
    const int kind = (d == 1) ? 3 : (k == 0) ? 0 : (k == d - 1) ? 2 : 1;
    hipError_t e = launch_laplacian_core(x->dtype, (const char*)x->data + (size_t)xo * esz, x->r[k], x->n[k],
                                         x->r[k + 1], kind, alpha, (char*)out->data + (size_t)yo * esz, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "laplacian");
    xo += x->r[k] * x->n[k] * x->r[k + 1];
    yo += yr[k] * x->n[k] * yr[k + 1];
  }
  for (int k = 0; k <= d; ++k) out->r[k] = yr[k];
  return TT_OK;
}

tt_status tt_krylov_laplacian(tt_ctx* c, int32_t m, tt_vec* a) {
  if (!c || m < 1 || !a) return fail(c, TT_EINVAL, "krylov: bad arguments");
  tt_status s;
  int64_t S = 0;
  for (int j = 0; j < m; ++j) {
    if ((s = check_vec(c, &a[j], "a", false)) != TT_OK) return s;
    if (!same_shape(a[j], a[0])) return fail(c, TT_EINVAL, "krylov: outputs differ in shape");
  }
  const tt_vec& s0 = a[0];
  const int d = s0.d;
  for (int k = 0; k < d; ++k) S += s0.n[k];
  for (int j = 0; j < m; ++j)
    if (a[j].capacity < S) return fail(c, TT_ECAPACITY, "krylov: output capacity below sum_k n_k");
  CallScope scope(c);
  const size_t mark = c->ws_off;
  struct Mark {
    tt_ctx* c;
    size_t off;
    ~Mark() { c->ws_off = off; }
  } wmark{c, mark};
  const size_t esz = elt_size(s0.dtype);
  // x (ones, then -Delta_d a_j with ranks 2 on interior bonds: at most 4 sum_k n_k elements)
  char* xbuf = (char*)ws_alloc(c, (size_t)4 * S * esz);
  double* nrm = (double*)dev_scratch(c, 8);
  if (!xbuf) return fail(c, TT_ECAPACITY, "workspace too small for the Krylov vector: need " + std::to_string(c->required));
  if (!nrm) return fail(c, TT_ENOMEM, "krylov buffers");
  hipError_t e;
  tt_vec x = s0;
  for (int k = 0; k <= d; ++k) x.r[k] = 1;
  x.data = xbuf;
  x.capacity = 4 * S;
  if ((e = launch_fill_const(s0.dtype, xbuf, S, 1.0, c->stream)) != hipSuccess) return hip_fail(c, e, "ones");
  static const double one = 1.0;
  for (int j = 0; j < m; ++j) {
    // a_j = x_j rounded to TT-rank one (accuracy 0, rank cap 1), then normalised
    tt_sum xs{1, &one, &x};
    std::vector<RJob> jobs(1);
    make_job(c, &xs, 0.0, 1, &a[j], jobs[0]);
    if ((s = round_jobs(c, jobs)) != TT_OK) return s;
    if (jobs[0].status != TT_OK) return fail(c, jobs[0].status, "krylov: output capacity");
    int64_t off = 0;
    for (int k = 0; k + 1 < d; ++k) off += a[j].r[k] * a[j].n[k] * a[j].r[k + 1];
    char* lastp = (char*)a[j].data + (size_t)off * esz;
    const int64_t last = a[j].r[d - 1] * a[j].n[d - 1];
    if ((e = launch_sumsq(s0.dtype, lastp, last, nrm, c->stream)) != hipSuccess) return hip_fail(c, e, "norm");
    if ((e = launch_scale(s0.dtype, lastp, last, nrm, c->stream)) != hipSuccess) return hip_fail(c, e, "scale");
    if (j + 1 < m) {
      // x_{j+1} = -Delta_d a_j
      int64_t xo = 0, yo = 0;
      for (int k = 0; k < d; ++k) {
        const int kind = (d == 1) ? 3 : (k == 0) ? 0 : (k == d - 1) ? 2 : 1;
        if ((e = launch_laplacian_core(s0.dtype, (const char*)a[j].data + (size_t)xo * esz, a[j].r[k], a[j].n[k],
                                       a[j].r[k + 1], kind, -1.0, xbuf + (size_t)yo * esz, c->stream)) != hipSuccess)
          return hip_fail(c, e, "laplacian");
        xo += a[j].r[k] * a[j].n[k] * a[j].r[k + 1];
        const int64_t y0 = (k == 0) ? 1 : 2 * a[j].r[k], y1 = (k == d - 1) ? 1 : 2 * a[j].r[k + 1];
        yo += y0 * a[j].n[k] * y1;
      }
      x.r[0] = x.r[d] = 1;
      for (int k = 1; k < d; ++k) x.r[k] = 2 * a[j].r[k];
    }
  }
  // a zero vector cannot be normalised: report it (the all-ones start and -Delta_d keep every a_j nonzero)
  double hn = 0.0;
  if ((s = read_doubles(c, nrm, &hn, 1)) != TT_OK) return s;
  if (!(hn > 0.0) || !std::isfinite(hn)) return fail(c, TT_EBREAKDOWN, "krylov: zero or non-finite vector");
  return TT_OK;
}

tt_status tt_loo(tt_ctx* c, int32_t m, const tt_vec* q, double* loo, double* gram) {
  if (!c || m < 1 || !q || !loo) return fail(c, TT_EINVAL, "loo: bad arguments");
  tt_status s;
  for (int i = 0; i < m; ++i) {
    if ((s = check_vec(c, &q[i], "q", true)) != TT_OK) return s;
    if (!same_shape(q[0], q[i])) return fail(c, TT_EINVAL, "loo: vectors differ in shape");
  }
  CallScope scope(c);
  double* Gq = (double*)dev_scratch(c, (size_t)m * m * 8);
  if (!Gq) return fail(c, TT_ENOMEM, "loo gram");
  for (int i = 0; i < m; ++i)
    if ((s = gram_row(c, i, m, q, Gq)) != TT_OK) return s;
  if (gram && (s = read_doubles(c, Gq, gram, (size_t)m * m)) != TT_OK) return s;
  return loo_from_gram(c, Gq, m, loo);
}

tt_status tt_orthogonalize_capacity(int32_t scheme, int32_t m, const tt_sum* a, int64_t rank_guard, int64_t* ranks,
                                    int64_t* sizes) {
  if (scheme < TT_CGS || scheme > TT_HOUSEHOLDER || m < 1 || !a) return TT_EINVAL;
  const tt_vec* s0 = (a[0].ncomp >= 1 && a[0].comp) ? &a[0].comp[0] : nullptr;
  if (!s0 || s0->d < 1 || s0->d > TT_MAXD) return TT_EINVAL;
  const int d = s0->d;
  for (int i = 0; i < m; ++i) {
    if (a[i].ncomp < 1 || !a[i].comp) return TT_EINVAL;
    for (int c = 0; c < a[i].ncomp; ++c) {
      const tt_vec& v = a[i].comp[c];
      if (v.d != d || v.r[0] != 1 || v.r[d] != 1) return TT_EINVAL;
      for (int k = 0; k < d; ++k)
        if (v.n[k] != s0->n[k] || v.n[k] < 1 || v.r[k] < 1) return TT_EINVAL;
    }
  }
  int64_t caps[TT_MAXD + 1];
  rank_caps(*s0, caps);
  auto capped = [&](int64_t* b) {
    for (int k = 0; k <= d; ++k) {
      int64_t v = std::min(b[k], caps[k]);
      if (rank_guard > 0) v = std::min(v, rank_guard);
      b[k] = (k == 0 || k == d) ? 1 : v;
    }
  };
  // S[k]: sum of the bounds of q_0..q_{i-1}; acc[k]: Gram's running sum of input
  // ranks; U[k]: sum of the bounds of the Householder vectors u_0..u_i.
  std::vector<int64_t> S(d + 1, 0), acc(d + 1, 0), U(d + 1, 0);
  for (int i = 0; i < m; ++i) {
    int64_t ra[TT_MAXD + 1], b[TT_MAXD + 1];
    for (int k = 0; k <= d; ++k) {
      ra[k] = 0;
      for (int c = 0; c < a[i].ncomp; ++c) ra[k] += a[i].comp[c].r[k];
    }
    if (scheme == TT_GRAM) {
      // q_i rounds sum_{k<=i} R^{-1}(k, i) a_k
      for (int k = 0; k <= d; ++k) b[k] = (acc[k] += ra[k]);
    } else if (scheme == TT_HOUSEHOLDER) {
      // rounded w = a~_i (a_i plus earlier reflections), then w and i canonical
      // terms, then u_i = that plus one; q_i = e_i reflected by u_0..u_i
      int64_t bw[TT_MAXD + 1], b1[TT_MAXD + 1], u[TT_MAXD + 1];
      for (int k = 0; k <= d; ++k) bw[k] = ra[k] + U[k];
      capped(bw);
      for (int k = 0; k <= d; ++k) b1[k] = bw[k] + i;
      capped(b1);
      for (int k = 0; k <= d; ++k) u[k] = b1[k] + 1;
      capped(u);
      for (int k = 0; k <= d; ++k) b[k] = 1 + (U[k] += u[k]);
    } else if (scheme == TT_CGS2 || scheme == TT_MGS2) {
      // second pass: the rounded first-pass vector (at most min(R1, caps)) plus the basis
      for (int k = 0; k <= d; ++k) b[k] = std::min(ra[k] + S[k], caps[k]) + S[k];
    } else {
      for (int k = 0; k <= d; ++k) b[k] = ra[k] + S[k];
    }
    capped(b);
    int64_t sz = 0;
    for (int k = 0; k < d; ++k) sz += b[k] * s0->n[k] * b[k + 1];
    if (ranks)
      for (int k = 0; k <= d; ++k) ranks[(size_t)i * (d + 1) + k] = b[k];
    if (sizes) sizes[i] = sz;
    for (int k = 0; k <= d; ++k) S[k] += b[k];
  }
  return TT_OK;
}

tt_status tt_cond(tt_ctx* c, int32_t m, const tt_sum* a, double* kappa, double* gram) {
  if (!c || m < 1 || !a || !kappa) return fail(c, TT_EINVAL, "cond: bad arguments");
  tt_status s;
  for (int i = 0; i < m; ++i) {
    if ((s = check_sum(c, &a[i], "a")) != TT_OK) return s;
    if (!same_shape(a[i].comp[0], a[0].comp[0])) return fail(c, TT_EINVAL, "cond: inputs differ in shape");
  }
  CallScope scope(c);
  double* G = (double*)dev_scratch(c, (size_t)m * m * 8);
  if (!G) return fail(c, TT_ENOMEM, "cond gram");
  // G(i, j) = <a_i, a_j>, j <= i, in one batched launch, then mirrored
  std::vector<tt_sum> xs, ys;
  std::vector<int32_t> idx;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      xs.push_back(a[i]);
      ys.push_back(a[j]);
      idx.push_back(i * m + j);
    }
  if ((s = dot_pairs_idx(c, (int)xs.size(), xs.data(), ys.data(), G, &idx)) != TT_OK) return s;
  hipError_t e = launch_sym_lower(G, m, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "cond sym");
  if (gram && (s = read_doubles(c, G, gram, (size_t)m * m)) != TT_OK) return s;
  std::vector<double> sig((size_t)m * (m + 1) / 2);
  if ((s = block_spectra(c, G, m, 0, sig.data())) != TT_OK) return s;
  for (int k = 1; k <= m; ++k) {
    const double* sk = sig.data() + (size_t)(k - 1) * k / 2;
    const double hi = sk[0], lo = sk[k - 1];
    kappa[k - 1] = lo > 0.0 ? std::sqrt(hi / lo) : INFINITY;
  }
  return TT_OK;
}

tt_status tt_orthogonalize(tt_ctx* c, tt_scheme scheme, int32_t m, const tt_sum* a, double delta, int64_t rank_guard,
                           tt_vec* q, double* R, double* loo, tt_ortho_stats* stats) {
  if (!c || m < 1 || !a || !q || !R) return fail(c, TT_EINVAL, "orthogonalize: bad arguments");
  if (scheme < TT_CGS || scheme > TT_HOUSEHOLDER) return fail(c, TT_EINVAL, "orthogonalize: unknown scheme");
  if (!(delta >= 0.0) || !std::isfinite(delta)) return fail(c, TT_EINVAL, "orthogonalize: delta must be >= 0");
  tt_status s;
  for (int i = 0; i < m; ++i) {
    if ((s = check_sum(c, &a[i], "a")) != TT_OK) return s;
    if (!same_shape(a[i].comp[0], a[0].comp[0])) return fail(c, TT_EINVAL, "orthogonalize: inputs differ in shape");
    if ((s = check_vec(c, &q[i], "q", false)) != TT_OK) return s;
    if (!same_shape(q[i], a[0].comp[0])) return fail(c, TT_EINVAL, "orthogonalize: q shape differs from inputs");
  }
  tt_ortho_stats st;
  std::memset(&st, 0, sizeof(st));
  st.q_pre_size = stats ? stats->q_pre_size : nullptr;
  CallScope scope(c);
  const size_t mark = c->ws_off;
  struct Mark {
    tt_ctx* c;
    size_t off;
    ~Mark() { c->ws_off = off; }
  } wmark{c, mark};
  const int d = a[0].comp[0].d;
  double* R1 = (double*)dev_scratch(c, (size_t)m * m * 8);   // column-major: R(j, i) at i*m + j
  double* R2 = (double*)dev_scratch(c, (size_t)m * m * 8);
  double* Gq = (double*)dev_scratch(c, (size_t)m * m * 8);
  double* dots = (double*)dev_scratch(c, (size_t)m * 8);
  double* neg = (double*)dev_scratch(c, (size_t)m * 8);
  double* nrm = (double*)dev_scratch(c, (size_t)m * 8);
  if (!R1 || !R2 || !Gq || !dots || !neg || !nrm) return fail(c, TT_ENOMEM, "orthogonalize buffers");
  hipError_t e;
  if ((e = hipMemsetAsync(R1, 0, (size_t)m * m * 8, c->stream)) != hipSuccess) return hip_fail(c, e, "memset");
  if ((e = hipMemsetAsync(R2, 0, (size_t)m * m * 8, c->stream)) != hipSuccess) return hip_fail(c, e, "memset");
  auto finish = [&](tt_status rs) {
    if (stats) *stats = st;
    return rs;
  };

  if (scheme == TT_HOUSEHOLDER) return finish(ortho_householder(c, m, a, delta, rank_guard, q, R1, R, loo, Gq, st));

  if (scheme == TT_GRAM) {
    // G(i, j) = <a_i, a_j>  (one batched launch), Cholesky, R^{-1}
    std::vector<tt_sum> xs, ys;
    std::vector<int32_t> idx;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j <= i; ++j) {
        xs.push_back(a[i]);
        ys.push_back(a[j]);
        idx.push_back(i * m + j);
      }
    double* G = (double*)dev_scratch(c, (size_t)m * m * 8);
    double* Rinv = (double*)dev_scratch(c, (size_t)m * m * 8);
    int32_t* info = (int32_t*)dev_scratch(c, 8);
    if (!G || !Rinv || !info) return finish(fail(c, TT_ENOMEM, "gram buffers"));
    if ((s = dot_pairs_idx(c, (int)xs.size(), xs.data(), ys.data(), G, &idx)) != TT_OK) return finish(s);
    if ((e = launch_sym_lower(G, m, c->stream)) != hipSuccess) return finish(hip_fail(c, e, "sym"));
    // The dots are FP64 for either dtype, but FP32-bulk inputs carry their
    // storage error of u_32 relative to each vector, so their Gram matrix is
    // known to that level only: the singularity test uses the storage precision.
    const double udot = (a[0].comp[0].dtype == TT_F64) ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
    if ((e = launch_cholinv(G, m, Rinv, info, udot, c->stream)) != hipSuccess) return finish(hip_fail(c, e, "cholesky"));
    int32_t* hinfo = (int32_t*)c->pin.alloc(8);
    if ((e = hipMemcpyAsync(hinfo, info, 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return finish(hip_fail(c, e, "info"));
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return finish(hip_fail(c, e, "sync"));
    if (*hinfo != 0)
      return finish(fail(c, TT_ENOTSPD, "Gram matrix not positive definite at pivot " + std::to_string(*hinfo)));
    // R = L^T in column-major == lower triangle of L in row-major
    if ((e = launch_tril(G, m, R1, c->stream)) != hipSuccess) return finish(hip_fail(c, e, "tril"));
    if ((s = read_doubles(c, R1, R, (size_t)m * m)) != TT_OK) return finish(s);
    std::vector<double> rinv((size_t)m * m);
    if ((s = read_doubles(c, Rinv, rinv.data(), rinv.size())) != TT_OK) return finish(s);
    // q_i = round( sum_{k<=i} R^{-1}(k, i) a_k ): m independent roundings, one batch
    std::vector<std::vector<double>> coefs(m);
    std::vector<std::vector<tt_vec>> comps(m);
    std::vector<RJob> jobs(m);
    std::vector<tt_sum> sums(m);
    for (int i = 0; i < m; ++i) {
      for (int k = 0; k <= i; ++k)
        for (int cc = 0; cc < a[k].ncomp; ++cc) {
          coefs[i].push_back(rinv[(size_t)k * m + i] * a[k].coef[cc]);
          comps[i].push_back(a[k].comp[cc]);
        }
      sums[i] = tt_sum{(int32_t)comps[i].size(), coefs[i].data(), comps[i].data()};
      make_job(c, &sums[i], delta, 0, &q[i], jobs[i]);
      const int64_t pre = max_bond(jobs[i].R, d);
      st.max_pre_rank = (int32_t)std::max<int64_t>(st.max_pre_rank, pre);
      if (st.q_pre_size) st.q_pre_size[i] = packed_size(a[0].comp[0], jobs[i].R);
      if (rank_guard > 0 && pre > rank_guard) {
        jobs.resize(i);
        st.m_reached = i;
        break;
      }
    }
    const bool guarded = (int)jobs.size() < m;
    if (!jobs.empty()) {
      if ((s = round_jobs_grouped(c, jobs)) != TT_OK) return finish(s);
      for (auto& jb : jobs) {
        if (jb.status != TT_OK) return finish(fail(c, jb.status, "gram: output capacity"));
        st.max_post_rank = (int32_t)std::max<int64_t>(st.max_post_rank, max_bond(jb.out->r, d));
      }
      st.rounds = (int32_t)jobs.size();
    }
    if (guarded) return finish(fail(c, TT_EGUARD, "pre-round rank exceeds the guard at vector " + std::to_string(st.m_reached)));
    st.m_reached = m;
    if (loo) {
      for (int i = 0; i < m; ++i)
        if ((s = gram_row(c, i, m, q, Gq)) != TT_OK) return finish(s);
      if ((s = loo_from_gram(c, Gq, m, loo)) != TT_OK) return finish(s);
    }
    return finish(TT_OK);
  }

  // ---- CGS, MGS, CGS2, MGS2
  const bool modified = (scheme == TT_MGS || scheme == TT_MGS2);
  const int passes = (scheme == TT_CGS2 || scheme == TT_MGS2) ? 2 : 1;
  static const double one = 1.0;
  tt_vec p1;                                 // rounded first-pass vector of the two-pass schemes
  std::memset(&p1, 0, sizeof(p1));
  for (int i = 0; i < m; ++i) {
    tt_sum src = a[i];
    for (int pass = 0; pass < passes; ++pass) {
      double* Rk = (pass == 0) ? R1 : R2;
      std::vector<double> coefs(src.coef, src.coef + src.ncomp);
      std::vector<tt_vec> comps(src.comp, src.comp + src.ncomp);
      if (i > 0) {
        std::vector<tt_sum> xs(i, src), ys(i);
        for (int j = 0; j < i; ++j) ys[j] = tt_sum{1, &one, &q[j]};
        if ((s = dot_pairs(c, i, xs.data(), ys.data(), dots)) != TT_OK) return finish(s);
        double* col = Rk + (size_t)i * m;
        if (modified) {
          if ((e = launch_mgs_correct(dots, Gq, m, i, col, neg, c->stream)) != hipSuccess)
            return finish(hip_fail(c, e, "mgs"));
        } else {
          if ((e = hipMemcpyAsync(col, dots, (size_t)i * 8, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
            return finish(hip_fail(c, e, "copy"));
          if ((e = launch_neg(dots, neg, i, c->stream)) != hipSuccess) return finish(hip_fail(c, e, "neg"));
        }
        std::vector<double> hneg(i);
        if ((s = read_doubles(c, neg, hneg.data(), i)) != TT_OK) return finish(s);
        for (int j = 0; j < i; ++j) {
          coefs.push_back(hneg[j]);
          comps.push_back(q[j]);
        }
      }
      tt_sum p{(int32_t)comps.size(), coefs.data(), comps.data()};
      RJob probe;
      make_job(c, &p, delta, 0, nullptr, probe);
      const int64_t pre = max_bond(probe.R, d);
      st.max_pre_rank = (int32_t)std::max<int64_t>(st.max_pre_rank, pre);
      if (rank_guard > 0 && pre > rank_guard) {
        st.m_reached = i;
        // R of the completed prefix (columns < i) is still returned
        if (passes == 2 && (e = launch_add(R1, R2, R1, m * m, c->stream)) != hipSuccess)
          return finish(hip_fail(c, e, "R1+R2"));
        if ((s = read_doubles(c, R1, R, (size_t)m * m)) != TT_OK) return finish(s);
        return finish(fail(c, TT_EGUARD, "pre-round rank " + std::to_string(pre) + " exceeds the guard at vector " +
                                             std::to_string(i)));
      }
      tt_vec* dest = &q[i];
      if (st.q_pre_size && pass + 1 == passes) st.q_pre_size[i] = packed_size(a[0].comp[0], probe.R);
      if (pass + 1 < passes) {
        // first pass of CGS2/MGS2: keep the rounded p_1 in the workspace
        p1 = q[i];
        const int64_t cap = tt_round_out_capacity(&p);
        c->ws_off = mark;   // the previous p_1 is no longer needed
        p1.data = ws_alloc(c, (size_t)cap * elt_size(p1.dtype));
        p1.capacity = cap;
        if (!p1.data)
          return finish(fail(c, TT_ECAPACITY, "workspace too small for p_1: need " + std::to_string(c->required)));
        dest = &p1;
      }
      if ((s = round_one(c, &p, delta, dest)) != TT_OK) return finish(s);
      ++st.rounds;
      st.max_post_rank = (int32_t)std::max<int64_t>(st.max_post_rank, max_bond(dest->r, d));
      src = tt_sum{1, &one, &p1};
    }
    // R(i, i) = ||p|| = ||last core|| (cores 0..d-2 are left-orthonormal); q_i = p / R(i, i)
    tt_vec& qi = q[i];
    int64_t off = 0;
    for (int k = 0; k + 1 < d; ++k) off += qi.r[k] * qi.n[k] * qi.r[k + 1];
    const int64_t last = qi.r[d - 1] * qi.n[d - 1];
    char* lastp = (char*)qi.data + (size_t)off * elt_size(qi.dtype);
    if ((e = launch_sumsq(qi.dtype, lastp, last, nrm + i, c->stream)) != hipSuccess)
      return finish(hip_fail(c, e, "norm"));
    double* Rfin = (passes == 2) ? R2 : R1;
    if ((e = hipMemcpyAsync(Rfin + (size_t)i * m + i, nrm + i, 8, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
      return finish(hip_fail(c, e, "diag"));
    double hn = 0.0;
    if ((s = read_doubles(c, nrm + i, &hn, 1)) != TT_OK) return finish(s);
    if (!(hn > 0.0)) {
      st.m_reached = i;
      return finish(fail(c, hn == 0.0 ? TT_EBREAKDOWN : TT_ENONFINITE,
                         "zero or non-finite norm after projection at vector " + std::to_string(i)));
    }
    if ((e = launch_scale(qi.dtype, lastp, last, nrm + i, c->stream)) != hipSuccess)
      return finish(hip_fail(c, e, "scale"));
    if ((s = gram_row(c, i, m, q, Gq)) != TT_OK) return finish(s);
    st.m_reached = i + 1;
  }
  if (passes == 2) {
    if ((e = launch_add(R1, R2, R1, m * m, c->stream)) != hipSuccess) return finish(hip_fail(c, e, "R1+R2"));
  }
  if ((s = read_doubles(c, R1, R, (size_t)m * m)) != TT_OK) return finish(s);
  if (loo && (s = loo_from_gram(c, Gq, m, loo)) != TT_OK) return finish(s);
  return finish(TT_OK);
}

}  // extern "C"

// ============================================================================
// Serving engine (continuous batching of Gram-Schmidt steps, Algorithms 1-4)
// ============================================================================
namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int scheme_passes(int s) { return (s == TT_CGS2 || s == TT_MGS2) ? 2 : 1; }
bool scheme_modified(int s) { return s == TT_MGS || s == TT_MGS2; }

// Packed size of a TT with bond ranks c_k = min(R_k, caps_k).
int64_t capped_size(const tt_vec& shape, const int64_t* R) {
  int64_t caps[TT_MAXD + 1];
  rank_caps(shape, caps);
  int64_t c[TT_MAXD + 1];
  for (int k = 0; k <= shape.d; ++k) c[k] = std::min(R[k], caps[k]);
  c[0] = c[shape.d] = 1;
  int64_t s = 0;
  for (int k = 0; k < shape.d; ++k) s += c[k] * shape.n[k] * c[k + 1];
  return s;
}

// Rank bounds of a request: first-pass sum w + basis, and second-pass sum
// p_1 + basis (p_1 itself capped).
void request_ranks(const tt_request* r, int64_t* R1, int64_t* R2) {
  const tt_vec& s0 = r->w.comp[0];
  const int d = s0.d;
  int64_t caps[TT_MAXD + 1];
  rank_caps(s0, caps);
  for (int k = 0; k <= d; ++k) {
    int64_t rw = 0, rq = 0;
    for (int i = 0; i < r->w.ncomp; ++i) rw += r->w.comp[i].r[k];
    for (int j = 0; j < r->b; ++j) rq += r->basis[j].r[k];
    R1[k] = (k == 0 || k == d) ? 1 : rw + rq;
    R2[k] = (k == 0 || k == d) ? 1 : std::min(R1[k], caps[k]) + rq;
  }
}

bool request_valid(const tt_request* r) {
  if (!r || r->scheme < TT_CGS || r->scheme > TT_MGS2 || r->b < 0 || (r->b > 0 && !r->basis)) return false;
  if (r->w.ncomp < 1 || !r->w.comp || !r->w.coef) return false;
  return true;
}

struct EngReq {
  int64_t id = 0;
  tt_request r;
  std::vector<tt_vec> basis;
  std::vector<double> wcoef;
  std::vector<tt_vec> wcomp;
  int passes = 1;
  bool modified = false;
  int stage = 0;                 // 0 dots (pass 1), 1 round (pass 1), 2 dots (pass 2), 3 round (pass 2), 4 normalise
  std::vector<double> rsum;      // column b of R, summed over the passes
  std::vector<double> rpass;     // coefficients of the current pass
  tt_vec p1;                     // first-pass result (in the request scratch)
  double* gram_dev = nullptr;    // basis Gram in the scratch (MGS), or null = identity
  int dtype = 0;
};

}  // namespace

struct tt_engine {
  tt_ctx* c = nullptr;
  int64_t next_id = 1;
  std::vector<EngReq*> live;
  std::vector<std::pair<int64_t, tt_status>> done;
};

extern "C" {

int64_t tt_request_out_capacity(const tt_request* r) {
  if (!request_valid(r)) return -1;
  int64_t R1[TT_MAXD + 1], R2[TT_MAXD + 1];
  request_ranks(r, R1, R2);
  return capped_size(r->w.comp[0], scheme_passes(r->scheme) == 2 ? R2 : R1);
}

int64_t tt_request_scratch_bytes(const tt_request* r) {
  if (!request_valid(r)) return -1;
  int64_t R1[TT_MAXD + 1], R2[TT_MAXD + 1];
  request_ranks(r, R1, R2);
  size_t bytes = 256;   // alignment slack
  if (scheme_modified(r->scheme) && r->b > 0) bytes += al256((size_t)r->b * r->b * 8);
  if (scheme_passes(r->scheme) == 2) bytes += al256((size_t)capped_size(r->w.comp[0], R1) * elt_size(r->w.comp[0].dtype));
  return (int64_t)bytes;
}

tt_status tt_engine_create(tt_ctx* c, tt_engine** e) {
  if (!c || !e) return TT_EINVAL;
  *e = new tt_engine();
  (*e)->c = c;
  return TT_OK;
}

void tt_engine_destroy(tt_engine* e) {
  if (!e) return;
  for (EngReq* q : e->live) delete q;
  delete e;
}

int32_t tt_engine_pending(const tt_engine* e) { return e ? (int32_t)(e->live.size() + e->done.size()) : 0; }

tt_status tt_engine_submit(tt_engine* e, const tt_request* r, int64_t* id) {
  if (!e || !id) return TT_EINVAL;
  tt_ctx* c = e->c;
  if (!request_valid(r)) return fail(c, TT_EINVAL, "engine: bad request");
  tt_status s;
  if ((s = check_sum(c, &r->w, "w")) != TT_OK) return s;
  const tt_vec& shape = r->w.comp[0];
  for (int j = 0; j < r->b; ++j) {
    if ((s = check_vec(c, &r->basis[j], "basis", true)) != TT_OK) return s;
    if (!same_shape(r->basis[j], shape)) return fail(c, TT_EINVAL, "engine: basis shape differs from w");
  }
  if ((s = check_vec(c, r->q_out, "q_out", false)) != TT_OK) return s;
  if (!same_shape(*r->q_out, shape)) return fail(c, TT_EINVAL, "engine: q_out shape differs from w");
  if (!r->r_out) return fail(c, TT_EINVAL, "engine: r_out is NULL");
  if (!(r->delta >= 0.0) || !std::isfinite(r->delta)) return fail(c, TT_EINVAL, "engine: delta must be >= 0");
  if (r->q_out->capacity < tt_request_out_capacity(r)) return fail(c, TT_ECAPACITY, "engine: q_out capacity");
  const int64_t need = tt_request_scratch_bytes(r);
  if (!r->scratch || r->scratch_bytes < need)
    return fail(c, TT_ECAPACITY, "engine: request scratch needs " + std::to_string(need) + " bytes");
  CallScope scope(c);
  EngReq* q = new EngReq();
  q->id = e->next_id++;
  q->r = *r;
  q->basis.assign(r->basis, r->basis + r->b);
  q->wcoef.assign(r->w.coef, r->w.coef + r->w.ncomp);
  q->wcomp.assign(r->w.comp, r->w.comp + r->w.ncomp);
  q->passes = scheme_passes(r->scheme);
  q->modified = scheme_modified(r->scheme);
  q->dtype = shape.dtype;
  q->rsum.assign(r->b, 0.0);
  char* base = (char*)(((uintptr_t)r->scratch + 255) & ~(uintptr_t)255);
  if (q->modified && r->b > 0 && r->basis_gram) {
    q->gram_dev = (double*)base;
    const size_t gb = (size_t)r->b * r->b * 8;
    double* h = (double*)c->pin.alloc(gb);
    if (!h) {
      delete q;
      return fail(c, TT_ENOMEM, "engine: staging");
    }
    std::memcpy(h, r->basis_gram, gb);
    hipError_t he = hipMemcpyAsync(q->gram_dev, h, gb, hipMemcpyHostToDevice, c->stream);
    if (he != hipSuccess) {
      delete q;
      return hip_fail(c, he, "engine: gram upload");
    }
  }
  if (q->modified && r->b > 0) base += al256((size_t)r->b * r->b * 8);
  if (q->passes == 2) {
    int64_t R1[TT_MAXD + 1], R2[TT_MAXD + 1];
    request_ranks(r, R1, R2);
    q->p1 = *r->q_out;
    q->p1.data = base;
    q->p1.capacity = capped_size(shape, R1);
  }
  e->live.push_back(q);
  *id = q->id;
  return TT_OK;
}

tt_status tt_engine_step(tt_engine* e, int32_t max_done, int64_t* done_ids, tt_status* done_status,
                         int32_t* ndone) {
  if (!e || !ndone || (max_done > 0 && (!done_ids || !done_status))) return TT_EINVAL;
  tt_ctx* c = e->c;
  CallScope scope(c);
  static const double one = 1.0;
  hipError_t he;
  tt_status s;
  auto finish_req = [&](EngReq* q, tt_status st) {
    e->done.emplace_back(q->id, st);
    q->stage = -1;
  };
  // source sum of the current pass: w, or the rounded first-pass vector
  auto src_sum = [&](EngReq* q) -> tt_sum {
    if (q->stage >= 2) return tt_sum{1, &one, &q->p1};
    return tt_sum{(int32_t)q->wcomp.size(), q->wcoef.data(), q->wcomp.data()};
  };
  std::vector<EngReq*> A, B, F;
  for (EngReq* q : e->live) {
    if (q->stage == 0 || q->stage == 2) A.push_back(q);
    else if (q->stage == 1 || q->stage == 3) B.push_back(q);
    else if (q->stage == 4) F.push_back(q);
  }
  for (int dt = 0; dt < 2; ++dt) {
    // ---- inner products <src, q_j> and projection coefficients of the pass
    std::vector<EngReq*> grp;
    for (EngReq* q : A)
      if (q->dtype == dt) grp.push_back(q);
    if (!grp.empty()) {
      std::vector<tt_sum> xs, ys;
      std::vector<size_t> off;
      for (EngReq* q : grp) {
        off.push_back(xs.size());
        const tt_sum src = src_sum(q);
        for (int j = 0; j < q->r.b; ++j) {
          xs.push_back(src);
          ys.push_back(tt_sum{1, &one, &q->basis[j]});
        }
      }
      const size_t np = xs.size();
      if (np > 0) {
        double* D = (double*)dev_scratch(c, np * 8);
        double* Rd = (double*)dev_scratch(c, np * 8);
        if (!D || !Rd) return fail(c, TT_ENOMEM, "engine: step buffers");
        if ((s = dot_pairs(c, (int)np, xs.data(), ys.data(), D)) != TT_OK) return s;
        std::vector<CoefTask> ct;
        for (size_t g = 0; g < grp.size(); ++g) {
          if (grp[g]->r.b == 0) continue;
          CoefTask t;
          t.dots = D + off[g];
          t.gram = grp[g]->gram_dev;
          t.r = Rd + off[g];
          t.b = grp[g]->r.b;
          t.modified = grp[g]->modified ? 1 : 0;
          ct.push_back(t);
        }
        const CoefTask* dct = upload(c, ct);
        if (!dct) return fail(c, TT_ENOMEM, "engine: task upload");
        if ((he = launch_coef_batched(dct, (int)ct.size(), c->stream)) != hipSuccess) return hip_fail(c, he, "coef");
        std::vector<double> hr(np);
        if ((s = read_doubles(c, Rd, hr.data(), np)) != TT_OK) return s;
        for (size_t g = 0; g < grp.size(); ++g) {
          EngReq* q = grp[g];
          q->rpass.assign(hr.begin() + off[g], hr.begin() + off[g] + q->r.b);
        }
      }
      for (EngReq* q : grp) {
        if (q->r.b == 0) q->rpass.clear();
        for (int j = 0; j < q->r.b; ++j) q->rsum[j] += q->rpass[j];
        q->stage += 1;
      }
    }
  }
  for (int dt = 0; dt < 2; ++dt) {
    // ---- rounding of the pass: round(src - sum_j r_j q_j)
    std::vector<EngReq*> grp;
    for (EngReq* q : B)
      if (q->dtype == dt) grp.push_back(q);
    if (grp.empty()) continue;
    std::vector<std::vector<double>> coefs(grp.size());
    std::vector<std::vector<tt_vec>> comps(grp.size());
    std::vector<tt_sum> sums(grp.size());
    std::vector<RJob> jobs;
    std::vector<EngReq*> jq;
    for (size_t g = 0; g < grp.size(); ++g) {
      EngReq* q = grp[g];
      const tt_sum src = src_sum(q);
      coefs[g].assign(src.coef, src.coef + src.ncomp);
      comps[g].assign(src.comp, src.comp + src.ncomp);
      for (int j = 0; j < q->r.b; ++j) {
        coefs[g].push_back(-q->rpass[j]);
        comps[g].push_back(q->basis[j]);
      }
      sums[g] = tt_sum{(int32_t)comps[g].size(), coefs[g].data(), comps[g].data()};
      tt_vec* dest = (q->stage == 1 && q->passes == 2) ? &q->p1 : q->r.q_out;
      RJob jb;
      make_job(c, &sums[g], q->r.delta, 0, dest, jb);
      std::vector<RJob> one_job(1, jb);
      if (round_workspace_bytes(one_job) < 0) {   // a shape the tile kernels do not support
        finish_req(q, TT_ENOTIMPL);
        continue;
      }
      jobs.push_back(jb);
      jq.push_back(q);
    }
    if (!jobs.empty()) {
      if ((s = round_jobs(c, jobs)) != TT_OK) return s;
      for (size_t i = 0; i < jobs.size(); ++i) {
        EngReq* q = jq[i];
        if (jobs[i].status != TT_OK) {
          finish_req(q, jobs[i].status);
          continue;
        }
        q->stage = (q->stage == 1 && q->passes == 2) ? 2 : 4;
      }
    }
  }
  if (!F.empty()) {
    // ---- R(b, b) = ||p|| = ||last core|| (cores 0..d-2 left-orthonormal), q = p / ||p||
    double* N = (double*)dev_scratch(c, F.size() * 8);
    if (!N) return fail(c, TT_ENOMEM, "engine: norms");
    std::vector<char*> lastp(F.size());
    std::vector<int64_t> lastn(F.size());
    for (size_t k = 0; k < F.size(); ++k) {
      tt_vec& qo = *F[k]->r.q_out;
      int64_t off = 0;
      for (int i = 0; i + 1 < qo.d; ++i) off += qo.r[i] * qo.n[i] * qo.r[i + 1];
      lastn[k] = qo.r[qo.d - 1] * qo.n[qo.d - 1];
      lastp[k] = (char*)qo.data + (size_t)off * elt_size(qo.dtype);
      if ((he = launch_sumsq(qo.dtype, lastp[k], lastn[k], N + k, c->stream)) != hipSuccess)
        return hip_fail(c, he, "engine: norm");
      if ((he = launch_scale(qo.dtype, lastp[k], lastn[k], N + k, c->stream)) != hipSuccess)
        return hip_fail(c, he, "engine: scale");
    }
    std::vector<double> hn(F.size());
    if ((s = read_doubles(c, N, hn.data(), F.size())) != TT_OK) return s;
    for (int dt = 0; dt < 2; ++dt) {
      std::vector<tt_sum> xs, ys;
      std::vector<std::pair<size_t, size_t>> where;   // (request, offset)
      for (size_t k = 0; k < F.size(); ++k) {
        EngReq* q = F[k];
        if (q->dtype != dt || !q->r.gram_out || !(hn[k] > 0.0)) continue;
        where.emplace_back(k, xs.size());
        for (int j = 0; j < q->r.b; ++j) {
          xs.push_back(tt_sum{1, &one, q->r.q_out});
          ys.push_back(tt_sum{1, &one, &q->basis[j]});
        }
      }
      if (xs.empty()) continue;
      double* G = (double*)dev_scratch(c, xs.size() * 8);
      if (!G) return fail(c, TT_ENOMEM, "engine: gram row");
      if ((s = dot_pairs(c, (int)xs.size(), xs.data(), ys.data(), G)) != TT_OK) return s;
      std::vector<double> hg(xs.size());
      if ((s = read_doubles(c, G, hg.data(), hg.size())) != TT_OK) return s;
      for (auto& w : where) {
        EngReq* q = F[w.first];
        std::copy(hg.begin() + w.second, hg.begin() + w.second + q->r.b, q->r.gram_out);
      }
    }
    for (size_t k = 0; k < F.size(); ++k) {
      EngReq* q = F[k];
      for (int j = 0; j < q->r.b; ++j) q->r.r_out[j] = q->rsum[j];
      q->r.r_out[q->r.b] = hn[k];
      if (hn[k] > 0.0) finish_req(q, TT_OK);
      else finish_req(q, hn[k] == 0.0 ? TT_EBREAKDOWN : TT_ENONFINITE);
    }
  }
  // retire finished requests, report up to max_done
  std::vector<EngReq*> keep;
  for (EngReq* q : e->live) {
    if (q->stage < 0) delete q;
    else keep.push_back(q);
  }
  e->live.swap(keep);
  int32_t n = 0;
  while (n < max_done && !e->done.empty()) {
    done_ids[n] = e->done.front().first;
    done_status[n] = e->done.front().second;
    e->done.erase(e->done.begin());
    ++n;
  }
  *ndone = n;
  return TT_OK;
}

}  // extern "C"
