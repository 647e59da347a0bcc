// Allocation-free TT inner product: tt_dot_noalloc of the C ABI.
//
// For callers that cannot allocate (code under HIP graph capture, tight serving
// loops): <x, y> of two TT-vectors with the contraction of tt_dot (dotk.h), its
// FP64 scratch taken from a fixed file-scope device array instead of a
// workspace, the pair's geometry passed by value as a kernel argument, and the
// result written to caller device memory.  The call issues one kernel launch on
// the caller's stream; it allocates nothing and does not synchronise.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/ttortho.h"
#include "common.h"
#include "dotk.h"

namespace tto {

namespace {

// Scratch of every tt_dot_noalloc call on a device: W (2 wcap doubles) and tmp.
// Each device holds its own copy from the first call until the process ends.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[NOALLOC_MAX_DEVICES] = {};   // device address of `scratch`, per device

// Address of this device's `scratch`, looked up once per device with that
// device current (the array's name is not a device address in host code).
hipError_t scratch_ptr(int dev, double** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = (double*)p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

struct DotArgs {
  int32_t d;
  const void* x;
  const void* y;
  double* w;
  int64_t wcap;
  double* tmp;
  double* out;
  int32_t n[TT_MAXD];
  int32_t rx[TT_MAXD + 1];
  int32_t ry[TT_MAXD + 1];
};

struct DotGeoArg {
  const DotArgs* a;
  __device__ int64_t n(int k) const { return a->n[k]; }
  __device__ int64_t x(int k) const { return a->rx[k]; }
  __device__ int64_t y(int k) const { return a->ry[k]; }
};

template <typename T>
__global__ __launch_bounds__(DOT_THREADS) void k_dot_args(const DotArgs args) {
  __shared__ double part[DOT_WAVES][256];
  const DotGeoArg g{&args};
  const double v = dot_pair<T>(g, args.d, args.x, args.y, args.w, args.wcap, args.tmp, part);
  if (threadIdx.x == 0) *args.out = v;
}

bool vec_ok(const tt_vec* v) {
  if (!v || v->d < 1 || v->d > TT_MAXD || !v->data) return false;
  if (v->dtype != TT_F64 && v->dtype != TT_F32) return false;
  if (v->r[0] != 1 || v->r[v->d] != 1) return false;
  int64_t size = 0;
  for (int k = 0; k < v->d; ++k) {
    if (v->n[k] < 1 || v->r[k] < 1 || v->n[k] > INT32_MAX || v->r[k] > INT32_MAX) return false;
    size += v->r[k] * v->n[k] * v->r[k + 1];
  }
  return size <= v->capacity;
}

}  // namespace

}  // namespace tto

extern "C" tt_status tt_dot_noalloc(void* stream, const tt_vec* x, const tt_vec* y, double* out) {
  using namespace tto;
  if (!vec_ok(x) || !vec_ok(y) || !out || x->d != y->d || x->dtype != y->dtype) return TT_EINVAL;
  for (int k = 0; k < x->d; ++k)
    if (x->n[k] != y->n[k]) return TT_EINVAL;
  int64_t wcap = 1, tcap = 1;
  for (int k = 0; k < x->d; ++k) {
    wcap = std::max(wcap, x->r[k + 1] * y->r[k + 1]);
    tcap = std::max(tcap, x->r[k] * x->n[k] * y->r[k + 1]);
  }
  const int64_t wpad = (2 * wcap + 31) & ~(int64_t)31;   // tmp starts 256 bytes aligned
  if ((size_t)(wpad + tcap) * sizeof(double) > NOALLOC_SCRATCH_BYTES) return TT_ECAPACITY;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return TT_EDEVICE;
  double* base = nullptr;
  if (scratch_ptr(dev, &base) != hipSuccess) return TT_EDEVICE;
  DotArgs a;
  std::memset(&a, 0, sizeof(a));
  a.d = x->d;
  a.x = x->data;
  a.y = y->data;
  a.w = base;
  a.wcap = wcap;
  a.tmp = base + wpad;
  a.out = out;
  for (int k = 0; k < x->d; ++k) a.n[k] = (int32_t)x->n[k];
  for (int k = 0; k <= x->d; ++k) {
    a.rx[k] = (int32_t)x->r[k];
    a.ry[k] = (int32_t)y->r[k];
  }
  const hipStream_t s = (hipStream_t)stream;
  if (x->dtype == TT_F64) hipLaunchKernelGGL(k_dot_args<double>, dim3(1), dim3(DOT_THREADS), 0, s, a);
  else hipLaunchKernelGGL(k_dot_args<float>, dim3(1), dim3(DOT_THREADS), 0, s, a);
  return hipGetLastError() == hipSuccess ? TT_OK : TT_EDEVICE;
}
