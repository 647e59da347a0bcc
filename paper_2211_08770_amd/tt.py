"""Thin Python binding of libttortho (argument marshalling only).

Every operation is one call into the C ABI declared in ``include/ttortho.h``;
PyTorch provides device memory and the stream.  The library is loaded on
first use and its absence is an error: there is no fallback path.

TT-vectors are :class:`TT` objects: one packed 1-D device tensor holding the
cores row-major ``[r_k][n_k][r_{k+1}]`` back to back, plus mode sizes and ranks.
A lazy sum is a list of ``(coef, TT)`` pairs.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np
import torch

__all__ = ["TT", "dot", "dot_batched", "axpy", "norm", "round", "round_batched", "round_randomized", "orthogonalize",
           "loo", "laplacian",
           "krylov_laplacian",
           "Engine", "TTError", "cond", "effective_delta", "BatchRounder", "library_path", "SCHEMES", "round_workspace_bytes", "round_out_capacity", "set_svd_block_min"]

TT_MAXD = 64
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libttortho.so"

SCHEMES = {"cgs": 0, "mgs": 1, "cgs2": 2, "mgs2": 3, "gram": 4, "householder": 5}
_F64, _F32 = 0, 1
_STATUS = {0: "TT_OK", -1: "TT_EINVAL", -2: "TT_ENOMEM", -3: "TT_ECAPACITY", -4: "TT_ENOTSPD",
           -5: "TT_EBREAKDOWN", -6: "TT_ENONFINITE", -7: "TT_EDEVICE", -8: "TT_EGUARD", -9: "TT_ENOTIMPL"}


class TTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = _STATUS.get(status, str(status))


class _Vec(C.Structure):
    _fields_ = [("d", C.c_int32), ("dtype", C.c_int32), ("n", C.c_int64 * TT_MAXD),
                ("r", C.c_int64 * (TT_MAXD + 1)), ("data", C.c_void_p), ("capacity", C.c_int64)]


class _Sum(C.Structure):
    _fields_ = [("ncomp", C.c_int32), ("coef", C.POINTER(C.c_double)), ("comp", C.POINTER(_Vec))]


class _Stats(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("m_reached", C.c_int32), ("max_pre_rank", C.c_int32),
                ("max_post_rank", C.c_int32), ("q_pre_size", C.POINTER(C.c_int64))]


class _Request(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("b", C.c_int32), ("basis", C.POINTER(_Vec)),
                ("basis_gram", C.POINTER(C.c_double)), ("w", _Sum), ("delta", C.c_double),
                ("q_out", C.POINTER(_Vec)), ("r_out", C.POINTER(C.c_double)), ("gram_out", C.POINTER(C.c_double)),
                ("scratch", C.c_void_p), ("scratch_bytes", C.c_int64)]


_lib = None
_lib_lock = threading.Lock()


def library_path() -> str:
    return os.path.join(_HERE, _LIBNAME)


def _load():
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2211_08770_amd.build`")
        lib = C.CDLL(path)
        P = C.c_void_p
        lib.tt_ctx_create.argtypes = [C.POINTER(P), C.c_int, P]
        lib.tt_ctx_create.restype = C.c_int
        lib.tt_ctx_destroy.argtypes = [P]
        lib.tt_ctx_set_workspace.argtypes = [P, P, C.c_size_t]
        lib.tt_ctx_set_workspace.restype = C.c_int
        lib.tt_ctx_required_bytes.argtypes = [P]
        lib.tt_ctx_required_bytes.restype = C.c_size_t
        lib.tt_last_error.argtypes = [P]
        lib.tt_last_error.restype = C.c_char_p
        lib.tt_status_str.argtypes = [C.c_int]
        lib.tt_status_str.restype = C.c_char_p
        lib.tt_dot_batched.argtypes = [P, C.c_int32, C.POINTER(_Sum), C.POINTER(_Sum), C.POINTER(C.c_double)]
        lib.tt_dot_batched.restype = C.c_int
        lib.tt_dot.argtypes = [P, C.POINTER(_Sum), C.POINTER(_Sum), C.POINTER(C.c_double)]
        lib.tt_dot.restype = C.c_int
        lib.tt_axpy.argtypes = [P, C.c_double, C.POINTER(_Vec), C.POINTER(_Vec), C.POINTER(_Vec)]
        lib.tt_axpy.restype = C.c_int
        lib.tt_round.argtypes = [P, C.POINTER(_Sum), C.c_double, C.c_int64, C.POINTER(_Vec), C.POINTER(C.c_double)]
        lib.tt_norm.argtypes = [P, C.POINTER(_Sum), C.POINTER(C.c_double)]
        lib.tt_norm.restype = C.c_int
        lib.tt_round.restype = C.c_int
        lib.tt_round_batched.argtypes = [P, C.c_int32, C.POINTER(_Sum), C.POINTER(C.c_double),
                                         C.POINTER(C.c_int64), C.POINTER(_Vec), C.POINTER(C.c_int)]
        lib.tt_round_batched.restype = C.c_int
        lib.tt_round_out_capacity.argtypes = [C.POINTER(_Sum)]
        lib.tt_round_out_capacity.restype = C.c_int64
        lib.tt_round_workspace_bytes.argtypes = [C.POINTER(_Sum)]
        lib.tt_round_workspace_bytes.restype = C.c_int64
        lib.tt_orthogonalize.argtypes = [P, C.c_int, C.c_int32, C.POINTER(_Sum), C.c_double, C.c_int64,
                                         C.POINTER(_Vec), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(_Stats)]
        lib.tt_orthogonalize.restype = C.c_int
        lib.tt_loo.argtypes = [P, C.c_int32, C.POINTER(_Vec), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.tt_loo.restype = C.c_int
        lib.tt_round_batched_async.argtypes = [P, C.c_int32, C.POINTER(_Sum), C.POINTER(C.c_double),
                                               C.POINTER(C.c_int64), C.POINTER(_Vec), C.c_void_p, C.c_void_p,
                                               C.c_void_p]
        lib.tt_round_batched_async.restype = C.c_int
        lib.tt_ctx_set_graphs.argtypes = [P, C.c_int]
        lib.tt_ctx_set_graphs.restype = C.c_int
        lib.tt_ctx_set_svd_block_min.argtypes = [P, C.c_int32]
        lib.tt_ctx_set_svd_block_min.restype = C.c_int
        lib.tt_ctx_graph_count.argtypes = [P]
        lib.tt_ctx_graph_count.restype = C.c_int32
        lib.tt_round_effective_delta.argtypes = [C.POINTER(_Sum), C.c_double]
        lib.tt_round_effective_delta.restype = C.c_double
        lib.tt_orthogonalize_capacity.argtypes = [C.c_int32, C.c_int32, C.POINTER(_Sum), C.c_int64,
                                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        lib.tt_orthogonalize_capacity.restype = C.c_int
        lib.tt_cond.argtypes = [P, C.c_int32, C.POINTER(_Sum), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.tt_cond.restype = C.c_int
        lib.tt_round_randomized.argtypes = [P, C.POINTER(_Sum), C.POINTER(_Vec), C.c_double, C.POINTER(_Vec)]
        lib.tt_round_randomized.restype = C.c_int
        lib.tt_laplacian.argtypes = [P, C.POINTER(_Vec), C.c_double, C.POINTER(_Vec)]
        lib.tt_laplacian.restype = C.c_int
        lib.tt_krylov_laplacian.argtypes = [P, C.c_int32, C.POINTER(_Vec)]
        lib.tt_krylov_laplacian.restype = C.c_int
        lib.tt_ctx_set_autotune.argtypes = [P, C.c_int]
        lib.tt_ctx_set_autotune.restype = C.c_int
        lib.tt_tune_tsqr.argtypes = [P, C.c_int64, C.c_int64, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        lib.tt_tune_tsqr.restype = C.c_int
        lib.tt_request_out_capacity.argtypes = [C.POINTER(_Request)]
        lib.tt_request_out_capacity.restype = C.c_int64
        lib.tt_request_scratch_bytes.argtypes = [C.POINTER(_Request)]
        lib.tt_request_scratch_bytes.restype = C.c_int64
        lib.tt_engine_create.argtypes = [P, C.POINTER(P)]
        lib.tt_engine_create.restype = C.c_int
        lib.tt_engine_destroy.argtypes = [P]
        lib.tt_engine_submit.argtypes = [P, C.POINTER(_Request), C.POINTER(C.c_int64)]
        lib.tt_engine_submit.restype = C.c_int
        lib.tt_engine_step.argtypes = [P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_int32)]
        lib.tt_engine_step.restype = C.c_int
        lib.tt_engine_pending.argtypes = [P]
        lib.tt_engine_pending.restype = C.c_int32
        _lib = lib
        return lib


class TT:
    """A TT-vector in packed device storage (cores row-major, back to back)."""

    def __init__(self, data: torch.Tensor, ns, ranks):
        self.data = data
        self.n = [int(v) for v in ns]
        self.r = [int(v) for v in ranks]
        if len(self.r) != len(self.n) + 1:
            raise ValueError("ranks must have d+1 entries")

    @property
    def d(self):
        return len(self.n)

    @property
    def dtype(self):
        return self.data.dtype

    def size(self):
        return sum(self.r[k] * self.n[k] * self.r[k + 1] for k in range(self.d))

    @classmethod
    def from_cores(cls, cores, device="cuda", dtype=None):
        ts = [torch.as_tensor(c) for c in cores]
        dt = dtype or ts[0].dtype
        flat = torch.cat([t.reshape(-1).to(dt) for t in ts]).to(device).contiguous()
        ns = [t.shape[1] for t in ts]
        ranks = [ts[0].shape[0]] + [t.shape[2] for t in ts]
        return cls(flat, ns, ranks)

    def cores(self):
        out, off = [], 0
        for k in range(self.d):
            sz = self.r[k] * self.n[k] * self.r[k + 1]
            out.append(self.data[off:off + sz].view(self.r[k], self.n[k], self.r[k + 1]))
            off += sz
        return out

    def numpy_cores(self):
        return [c.detach().cpu().numpy() for c in self.cores()]

    def _vec(self) -> _Vec:
        if self.data.dtype not in (torch.float64, torch.float32):
            raise TypeError("TT data must be float64 or float32")
        if not self.data.is_cuda or not self.data.is_contiguous():
            raise ValueError("TT data must be a contiguous device tensor")
        v = _Vec()
        v.d = self.d
        v.dtype = _F64 if self.data.dtype == torch.float64 else _F32
        for k, n in enumerate(self.n):
            v.n[k] = n
        for k, r in enumerate(self.r):
            v.r[k] = r
        v.data = self.data.data_ptr()
        v.capacity = self.data.numel()
        return v


def _as_terms(x):
    if isinstance(x, TT):
        return [(1.0, x)]
    return [(float(a), t) for a, t in x]


class _SumHolder:
    """Keeps the ctypes arrays of a lazy sum alive for the duration of a call."""

    def __init__(self, x):
        terms = _as_terms(x)
        self.tts = [t for _, t in terms]
        self.coef = (C.c_double * len(terms))(*[a for a, _ in terms])
        self.vecs = (_Vec * len(terms))(*[t._vec() for t in self.tts])
        self.s = _Sum(len(terms), self.coef, self.vecs)


class _Ctx:
    def __init__(self, device: int):
        self.lib = _load()
        self.device = device
        h = C.c_void_p()
        st = self.lib.tt_ctx_create(C.byref(h), device, C.c_void_p(torch.cuda.current_stream(device).cuda_stream))
        if st != 0:
            raise TTError(st, "tt_ctx_create failed")
        self.h = h
        self.ws = None
        self.ws_bytes = 0

    def ensure_ws(self, nbytes: int):
        if nbytes <= self.ws_bytes:
            return
        nbytes = int(nbytes * 1.25) + (1 << 20)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        self.ws_bytes = nbytes
        st = self.lib.tt_ctx_set_workspace(self.h, C.c_void_p(self.ws.data_ptr()), nbytes)
        if st != 0:
            raise TTError(st, "set_workspace failed")

    def check(self, st):
        if st != 0:
            raise TTError(st, self.lib.tt_last_error(self.h).decode())

    def call_with_ws(self, fn):
        """Run fn(); when it reports TT_ECAPACITY for the workspace, grow it and run fn again.
        A call whose later steps need more than its earlier ones (ranks that grow along a
        Gram-Schmidt run) reports only what it needed up to where it stopped, so the
        workspace grows with headroom (1.5 times the report) to keep the reruns few."""
        for _ in range(10):
            st = fn()
            if st == -3:
                need = int(self.lib.tt_ctx_required_bytes(self.h))
                if need > self.ws_bytes:
                    self.ensure_ws(need + need // 2)
                    continue
            self.check(st)
            return
        self.check(st)


_ctxs = {}


def _ctx(device=None) -> _Ctx:
    dev = torch.cuda.current_device() if device is None else int(device)
    stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev, stream)
    if key not in _ctxs:
        _ctxs[key] = _Ctx(dev)
    return _ctxs[key]


def _device_of(x):
    return _as_terms(x)[0][1].data.device.index


def dot(x, y) -> float:
    """<x, y> of two TT-vectors or lazy sums."""
    return dot_batched([(x, y)])[0]


def dot_batched(pairs):
    if not pairs:
        return np.zeros(0)
    ctx = _ctx(_device_of(pairs[0][0]))
    hx = [_SumHolder(x) for x, _ in pairs]
    hy = [_SumHolder(y) for _, y in pairs]
    xs = (_Sum * len(pairs))(*[h.s for h in hx])
    ys = (_Sum * len(pairs))(*[h.s for h in hy])
    out = (C.c_double * len(pairs))()
    ctx.ensure_ws(64 << 20)
    ctx.call_with_ws(lambda: ctx.lib.tt_dot_batched(ctx.h, len(pairs), xs, ys, out))
    return np.array(out[:], dtype=np.float64)


def axpy(alpha: float, x: TT, y: TT) -> TT:
    """z = alpha * x + y (materialised TT sum, ranks add)."""
    ctx = _ctx(x.data.device.index)
    ranks = [1] + [a + b for a, b in zip(x.r[1:-1], y.r[1:-1])] + [1]
    size = sum(ranks[k] * x.n[k] * ranks[k + 1] for k in range(x.d))
    z = TT(torch.empty(size, dtype=x.dtype, device=x.data.device), x.n, ranks)
    vx, vy, vz = x._vec(), y._vec(), z._vec()
    ctx.check(ctx.lib.tt_axpy(ctx.h, float(alpha), C.byref(vx), C.byref(vy), C.byref(vz)))
    z.r = [int(vz.r[k]) for k in range(x.d + 1)]
    return z


def round_randomized(x, sketch: TT, delta: float = 0.0):
    """Randomize-then-Orthogonalize rounding of a TT or lazy sum with the given Gaussian sketch TT
    (FP64); delta > 0 rounds the result deterministically afterwards."""
    h = _SumHolder(x)
    first = h.tts[0]
    ctx = _ctx(first.data.device.index)
    d = first.d
    p = [1] * (d + 1)
    for k in range(1, d):
        p[k] = min(sketch.r[k], p[k - 1] * first.n[k - 1])
    cap = sum(p[k] * first.n[k] * p[k + 1] for k in range(d))
    if d == 1:
        cap = first.n[0]
    out = TT(torch.empty(max(cap, 1), dtype=first.dtype, device=first.data.device), first.n, [1] * (d + 1))
    vo = out._vec()
    vs = sketch._vec()
    ctx.ensure_ws(64 << 20)
    ctx.call_with_ws(lambda: ctx.lib.tt_round_randomized(ctx.h, C.byref(h.s), C.byref(vs), float(delta), C.byref(vo)))
    return _finish_out(out, vo)


def laplacian(x: TT, alpha: float = 1.0) -> TT:
    """alpha * Delta_d x (Dirichlet Laplacian as a rank-two TT-matrix; interior ranks double)."""
    ctx = _ctx(x.data.device.index)
    ranks = [1] + [2 * r for r in x.r[1:-1]] + [1]
    size = sum(ranks[k] * x.n[k] * ranks[k + 1] for k in range(x.d))
    y = TT(torch.empty(size, dtype=x.dtype, device=x.data.device), x.n, ranks)
    vx, vy = x._vec(), y._vec()
    ctx.check(ctx.lib.tt_laplacian(ctx.h, C.byref(vx), float(alpha), C.byref(vy)))
    y.r = [int(vy.r[k]) for k in range(x.d + 1)]
    return y


def krylov_laplacian(ns, m: int, dtype=torch.float64, device=None):
    """The m rank-one Krylov inputs of the paper's experiments (ones, -Delta_d, rank-one rounding)."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    ctx = _ctx(dev.index)
    size = int(sum(ns))
    A = [TT(torch.empty(size, dtype=dtype, device=dev), list(ns), [1] * (len(ns) + 1)) for _ in range(m)]
    va = (_Vec * m)(*[a._vec() for a in A])
    ctx.ensure_ws(64 << 20)
    ctx.call_with_ws(lambda: ctx.lib.tt_krylov_laplacian(ctx.h, m, va))
    return [_finish_out(a, va[i]) for i, a in enumerate(A)]


def round_out_capacity(x) -> int:
    h = _SumHolder(x)
    return int(_load().tt_round_out_capacity(C.byref(h.s)))


def effective_delta(x, delta: float) -> float:
    """delta_eff of tt_round_effective_delta: the accuracy TT-round guarantees for x
    (delta in FP64; at least the FP32 resolution of the merged cores in FP32-bulk)."""
    h = _SumHolder(x)
    return float(_load().tt_round_effective_delta(C.byref(h.s), float(delta)))


def round_workspace_bytes(x) -> int:
    h = _SumHolder(x)
    return int(_load().tt_round_workspace_bytes(C.byref(h.s)))


def _new_out(x):
    first = _as_terms(x)[0][1]
    cap = max(round_out_capacity(x), 1)
    return TT(torch.empty(cap, dtype=first.dtype, device=first.data.device), first.n, [1] * (first.d + 1))


def _packed(data: torch.Tensor, size: int) -> torch.Tensor:
    """The first `size` elements of an output buffer.  Output buffers are sized for the rank
    bounds; when the result is far smaller, it gets a buffer of its own so that keeping the
    result does not keep the bound-sized buffer alive."""
    if data.numel() > 2 * size + (1 << 16):
        return data[:size].clone()
    return data[:size]


def _finish_out(out: TT, v: _Vec):
    out.r = [int(v.r[k]) for k in range(out.d + 1)]
    out.data = _packed(out.data, out.size())
    return out


def set_autotune(on: bool = True, device=None):
    """Let TT-round time candidate TSQR tree shapes for unseen QR shapes (kept for the process)."""
    ctx = _ctx(device)
    ctx.check(ctx.lib.tt_ctx_set_autotune(ctx.h, 1 if on else 0))


def set_svd_block_min(rows: int, device=None):
    """R factors of more than `rows` rows (32..1024) take the block Jacobi SVD over many
    workgroups instead of the one-workgroup Jacobi (tt_ctx_set_svd_block_min)."""
    ctx = _ctx(device)
    ctx.check(ctx.lib.tt_ctx_set_svd_block_min(ctx.h, int(rows)))


def tune_tsqr(rows: int, cols: int, dtype=torch.float64, device=None):
    """Tune the TSQR tree shape of one QR shape class now; returns (leaf_rows, fanin)."""
    ctx = _ctx(device)
    lr, fi = C.c_int32(0), C.c_int32(0)
    ctx.ensure_ws(3 * rows * cols * (8 if dtype == torch.float64 else 4) + (1 << 20))
    ctx.call_with_ws(lambda: ctx.lib.tt_tune_tsqr(ctx.h, int(rows), int(cols), _F64 if dtype == torch.float64 else _F32,
                                                  C.byref(lr), C.byref(fi)))
    return lr.value, fi.value


def norm(x) -> float:
    """||x|| of a TT or lazy sum by the right-to-left QR sweep (no cancellation)."""
    h = _SumHolder(x)
    ctx = _ctx(h.tts[0].data.device.index)
    out = C.c_double(0.0)
    ws = int(ctx.lib.tt_round_workspace_bytes(C.byref(h.s)))
    if ws < 0:
        ctx.check(-9)
    ctx.ensure_ws(ws)
    ctx.call_with_ws(lambda: ctx.lib.tt_norm(ctx.h, C.byref(h.s), C.byref(out)))
    return out.value


def round(x, delta: float, max_rank: int = 0, return_norm: bool = False):
    """TT-round(x, delta): ||x - x~|| <= delta ||x||; x is a TT or a lazy sum."""
    h = _SumHolder(x)
    ctx = _ctx(h.tts[0].data.device.index)
    out = _new_out(x)
    vo = out._vec()
    nrm = C.c_double(0.0)
    ws = int(ctx.lib.tt_round_workspace_bytes(C.byref(h.s)))
    if ws < 0:
        ctx.check(-9)
    ctx.ensure_ws(ws)
    ctx.call_with_ws(lambda: ctx.lib.tt_round(ctx.h, C.byref(h.s), float(delta), int(max_rank), C.byref(vo),
                                              C.byref(nrm)))
    out = _finish_out(out, vo)
    return (out, nrm.value) if return_norm else out


def round_batched(xs, deltas, max_ranks=None, plan="host"):
    """Independent roundings of several TTs / lazy sums in shared launches.

    plan="host": tt_round_batched (each left-to-right step planned at the rank the device
    chose, read back by the host).  plan="bounds": tt_round_batched_async (every step planned
    at the rank bounds, no host synchronisation until the end), then the stream is synchronised
    and the ranks and statuses are read from pinned memory.
    """
    if plan == "bounds":
        return _round_batched_bounds(xs, deltas, max_ranks)
    n = len(xs)
    hs = [_SumHolder(x) for x in xs]
    ctx = _ctx(hs[0].tts[0].data.device.index)
    outs = [_new_out(x) for x in xs]
    vos = (_Vec * n)(*[o._vec() for o in outs])
    sums = (_Sum * n)(*[h.s for h in hs])
    if np.isscalar(deltas):
        deltas = [deltas] * n
    dl = (C.c_double * n)(*[float(v) for v in deltas])
    mr = (C.c_int64 * n)(*([int(v) for v in max_ranks] if max_ranks is not None else [0] * n))
    st = (C.c_int * n)()
    ws = sum(max(int(ctx.lib.tt_round_workspace_bytes(C.byref(h.s))), 0) for h in hs)
    ctx.ensure_ws(ws)
    ctx.call_with_ws(lambda: ctx.lib.tt_round_batched(ctx.h, n, sums, dl, mr, vos, st))
    return [_finish_out(o, vos[i]) for i, o in enumerate(outs)]


def _round_batched_bounds(xs, deltas, max_ranks=None):
    n = len(xs)
    hs = [_SumHolder(x) for x in xs]
    ctx = _ctx(hs[0].tts[0].data.device.index)
    outs = [_new_out(x) for x in xs]
    vos = (_Vec * n)(*[o._vec() for o in outs])
    sums = (_Sum * n)(*[h.s for h in hs])
    if np.isscalar(deltas):
        deltas = [deltas] * n
    dl = (C.c_double * n)(*[float(v) for v in deltas])
    mr = (C.c_int64 * n)(*([int(v) for v in max_ranks] if max_ranks is not None else [0] * n))
    ranks = torch.zeros(n * (TT_MAXD + 1), dtype=torch.int32, pin_memory=True)
    status = torch.full((n,), -99, dtype=torch.int32, pin_memory=True)
    ws = sum(max(int(ctx.lib.tt_round_workspace_bytes(C.byref(h.s))), 0) for h in hs)
    ctx.ensure_ws(ws)
    ctx.call_with_ws(lambda: ctx.lib.tt_round_batched_async(ctx.h, n, sums, dl, mr, vos, C.c_void_p(ranks.data_ptr()),
                                                             C.c_void_p(status.data_ptr()), None))
    torch.cuda.current_stream(ctx.device).synchronize()
    st = status.tolist()
    rk = ranks.view(n, TT_MAXD + 1).tolist()
    for j, o in enumerate(outs):
        if st[j] != 0:
            raise TTError(st[j], f"job {j} failed")
        o.r = [int(v) for v in rk[j][: o.d + 1]]
        o.data = _packed(o.data, o.size())
    return outs


class BatchRounder:
    """Repeated roundings of same-shaped inputs that stay in the same buffers (a solver loop):
    tt_round_batched_async on a stream of its own, with graph replay on (tt_ctx_set_graphs),
    so the first run() is captured and later ones launch the graph.  The outputs and the pinned
    rank/status arrays are allocated once; results() waits for the stream and returns the TTs."""

    def __init__(self, xs, deltas, max_ranks=None, graphs=True):
        self.n = n = len(xs)
        self.hs = [_SumHolder(x) for x in xs]
        dev = self.hs[0].tts[0].data.device
        self.stream = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(self.stream):
            self.ctx = _ctx(dev.index)
        self.ctx.check(self.ctx.lib.tt_ctx_set_graphs(self.ctx.h, 1 if graphs else 0))
        self.outs = [_new_out(x) for x in xs]
        self.cap = [o.data for o in self.outs]
        self.vos = (_Vec * n)(*[o._vec() for o in self.outs])
        self.sums = (_Sum * n)(*[h.s for h in self.hs])
        if np.isscalar(deltas):
            deltas = [deltas] * n
        self.dl = (C.c_double * n)(*[float(v) for v in deltas])
        self.mr = (C.c_int64 * n)(*([int(v) for v in max_ranks] if max_ranks is not None else [0] * n))
        self.ranks = torch.zeros(n * (TT_MAXD + 1), dtype=torch.int32, pin_memory=True)
        self.status = torch.full((n,), -99, dtype=torch.int32, pin_memory=True)
        ws = sum(max(int(self.ctx.lib.tt_round_workspace_bytes(C.byref(h.s))), 0) for h in self.hs)
        self.ctx.ensure_ws(2 * ws)

    def run(self):
        """Enqueue one rounding of every input (after the work of the current stream)."""
        self.stream.wait_stream(torch.cuda.current_stream(self.stream.device))
        c = self.ctx
        c.call_with_ws(lambda: c.lib.tt_round_batched_async(c.h, self.n, self.sums, self.dl, self.mr, self.vos,
                                                            C.c_void_p(self.ranks.data_ptr()),
                                                            C.c_void_p(self.status.data_ptr()), None))

    def graph_count(self):
        return int(self.ctx.lib.tt_ctx_graph_count(self.ctx.h))

    def results(self):
        self.stream.synchronize()
        st = self.status.tolist()
        rk = self.ranks.view(self.n, TT_MAXD + 1).tolist()
        out = []
        for j, o in enumerate(self.outs):
            if st[j] != 0:
                raise TTError(st[j], f"job {j} failed")
            t = TT(self.cap[j], o.n, [int(v) for v in rk[j][: o.d + 1]])
            t.data = t.data[: t.size()]
            out.append(t)
        return out


def q_rank_bounds(scheme: str, ra, ns, rank_guard: int = 0):
    """Upper bounds of the bond ranks of every q_i an orthogonalization returns
    (its output capacity), from tt_orthogonalize_capacity of the C ABI.

    ra[i][k]: summed component ranks of input i at bond k; ns: mode sizes.
    """
    lib = _load()
    d, m = len(ns), len(ra)
    vecs = (_Vec * m)()
    one = (C.c_double * 1)(1.0)
    sums = (_Sum * m)()
    for i in range(m):
        v = vecs[i]
        v.d, v.dtype = d, _F64
        for k in range(d):
            v.n[k] = int(ns[k])
        for k in range(d + 1):
            v.r[k] = 1 if k in (0, d) else int(ra[i][k])   # summed ranks: the boundary bonds count components
        sums[i] = _Sum(1, one, C.cast(C.byref(vecs, i * C.sizeof(_Vec)), C.POINTER(_Vec)))
    out = (C.c_int64 * (m * (d + 1)))()
    st = lib.tt_orthogonalize_capacity(SCHEMES[scheme], m, sums, int(rank_guard), out, None)
    if st != 0:
        raise TTError(st, "orthogonalize capacity: bad shapes")
    return [[int(out[i * (d + 1) + k]) for k in range(d + 1)] for i in range(m)]


def orthogonalize(scheme: str, A, delta: float, rank_guard: int = 0, with_loo: bool = True, q_capacity=None,
                  partial_on_guard: bool = False):
    """Q, R (and the LOO curve) of the TT vectors / lazy sums A (Algorithms 1-8).

    With partial_on_guard, a stop at the rank guard returns the completed
    prefix (Q[:m_reached], R with its columns from m_reached on set to zero, None,
    stats with "guard": True) instead of raising.
    """
    m = len(A)
    hs = [_SumHolder(a) for a in A]
    first = hs[0].tts[0]
    ctx = _ctx(first.data.device.index)
    sums = (_Sum * m)(*[h.s for h in hs])
    d = first.d
    ra = [[sum(t.r[k] for t in h.tts) for k in range(d + 1)] for h in hs]
    bounds = q_rank_bounds(scheme, ra, first.n, rank_guard)
    sizes = [sum(b[k] * first.n[k] * b[k + 1] for k in range(d)) for b in bounds]
    if scheme == "gram" and rank_guard > 0:
        # TT-Gram rounds q_i from the sum of a_1..a_i: its pre-round rank is known here, and a
        # q_i past the guard is never formed (one element of output is enough for it)
        run = [0] * (d + 1)
        for i, r in enumerate(ra):
            run = [x + y for x, y in zip(run, r)]
            if max(run[1:d]) > rank_guard:
                sizes[i] = 1
    if q_capacity is not None:
        sizes = [min(sz, int(q_capacity)) for sz in sizes]
    Q = [TT(torch.empty(max(sz, 1), dtype=first.dtype, device=first.data.device), first.n, [1] * (d + 1))
         for sz in sizes]
    vq = (_Vec * m)(*[q._vec() for q in Q])
    R = (C.c_double * (m * m))()
    L = (C.c_double * m)()
    stats = _Stats()
    pre_size = (C.c_int64 * m)()
    stats.q_pre_size = C.cast(pre_size, C.POINTER(C.c_int64))
    ctx.ensure_ws(256 << 20)
    call = lambda: ctx.lib.tt_orthogonalize(ctx.h, SCHEMES[scheme], m, sums, float(delta), int(rank_guard), vq, R,
                                            L if with_loo else None, C.byref(stats))
    if partial_on_guard:
        guarded = []

        def call_guard():
            st = call()
            if st == -8:
                guarded.append(True)
                return 0
            return st
        ctx.call_with_ws(call_guard)
        if guarded:
            k = stats.m_reached
            Qp = [_finish_out(Q[i], vq[i]) for i in range(k)]
            Rm = np.array(R[:], dtype=np.float64).reshape(m, m).T.copy()
            Rm[:, k:] = 0.0   # only the columns of the completed vectors are defined
            return Qp, Rm, None, {"rounds": stats.rounds, "m_reached": k, "max_pre_rank": stats.max_pre_rank,
                                  "max_post_rank": stats.max_post_rank, "guard": True}
    else:
        ctx.call_with_ws(call)
    Q = [_finish_out(q, vq[i]) for i, q in enumerate(Q)]
    Rm = np.array(R[:], dtype=np.float64).reshape(m, m).T.copy()   # column-major -> R[j, i]
    st = {"rounds": stats.rounds, "m_reached": stats.m_reached, "max_pre_rank": stats.max_pre_rank,
          "max_post_rank": stats.max_post_rank,
          # compression gain of q_i (Section 2): storage of the rounded lazy sum over that of q_i
          "gain": [int(pre_size[i]) / max(q.size(), 1) for i, q in enumerate(Q)]}
    return Q, Rm, (np.array(L[:]) if with_loo else None), st


def loo(Q):
    """||I_k - Q_k^T Q_k||_2 for k = 1..m and the Gram matrix Q^T Q."""
    m = len(Q)
    ctx = _ctx(Q[0].data.device.index)
    vq = (_Vec * m)(*[q._vec() for q in Q])
    out = (C.c_double * m)()
    G = (C.c_double * (m * m))()
    ctx.ensure_ws(64 << 20)
    ctx.call_with_ws(lambda: ctx.lib.tt_loo(ctx.h, m, vq, out, G))
    return np.array(out[:]), np.array(G[:]).reshape(m, m)


def cond(A):
    """kappa(A_k) = sqrt(kappa(G_k)), k = 1..m, from the FP64 Gram matrix of the
    TT-vectors or lazy sums A (tt_cond), and that Gram matrix."""
    m = len(A)
    ctx = _ctx(_device_of(A[0]))
    hs = [_SumHolder(a) for a in A]
    xs = (_Sum * m)(*[h.s for h in hs])
    out = (C.c_double * m)()
    G = (C.c_double * (m * m))()
    ctx.ensure_ws(64 << 20)
    ctx.call_with_ws(lambda: ctx.lib.tt_cond(ctx.h, m, xs, out, G))
    return np.array(out[:]), np.array(G[:]).reshape(m, m)


class Engine:
    """Continuous-batching engine of Gram-Schmidt steps (tt_engine_* of the C ABI).

    submit() hands one request -- orthogonalise the lazy sum ``w`` against an
    orthonormal resident ``basis`` with ``scheme`` -- and returns its id; each
    step() advances every request in flight by one stage and returns the
    requests that completed, as ``{id: (status, q, r, gram_row)}``.
    """

    def __init__(self, device=None):
        self.ctx = _ctx(device)
        h = C.c_void_p()
        self.ctx.check(self.ctx.lib.tt_engine_create(self.ctx.h, C.byref(h)))
        self.h = h
        self.inflight = {}

    def __del__(self):
        try:
            self.ctx.lib.tt_engine_destroy(self.h)
        except Exception:
            pass

    @staticmethod
    def _request(scheme, basis, basis_gram, w, delta):
        hb = [t._vec() for t in basis]
        hw = _SumHolder(w)
        req = _Request()
        req.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        req.b = len(basis)
        keep = {"w": hw}
        if basis:
            arr = (_Vec * len(hb))(*hb)
            keep["basis"] = arr
            req.basis = C.cast(arr, C.POINTER(_Vec))
        if basis_gram is not None and basis:
            g = np.ascontiguousarray(np.asarray(basis_gram, dtype=np.float64).reshape(len(basis), len(basis)))
            keep["gram"] = g
            req.basis_gram = g.ctypes.data_as(C.POINTER(C.c_double))
        req.w = hw.s
        req.delta = float(delta)
        return req, keep

    def footprint(self, scheme, basis, w, delta=0.0):
        """Device bytes a request holds while in flight: output TT and scratch."""
        req, keep = self._request(scheme, basis, None, w, delta)
        first = _as_terms(w)[0][1]
        elt = first.data.element_size()
        return int(self.ctx.lib.tt_request_out_capacity(C.byref(req))) * elt + \
            int(self.ctx.lib.tt_request_scratch_bytes(C.byref(req)))

    def submit(self, scheme, basis, w, delta, basis_gram=None, want_gram=True):
        req, keep = self._request(scheme, basis, basis_gram, w, delta)
        first = _as_terms(w)[0][1]
        cap = int(self.ctx.lib.tt_request_out_capacity(C.byref(req)))
        nbytes = int(self.ctx.lib.tt_request_scratch_bytes(C.byref(req)))
        if cap < 0 or nbytes < 0:
            raise TTError(-1, "bad request")
        q = TT(torch.empty(max(cap, 1), dtype=first.dtype, device=first.data.device), first.n, [1] * (first.d + 1))
        qv = q._vec()
        scratch = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=first.data.device)
        r = (C.c_double * (len(basis) + 1))()
        g = (C.c_double * max(len(basis), 1))()
        req.q_out = C.pointer(qv)
        req.r_out = r
        req.gram_out = g if want_gram else None
        req.scratch = scratch.data_ptr()
        req.scratch_bytes = scratch.numel()
        rid = C.c_int64(0)
        self.ctx.check(self.ctx.lib.tt_engine_submit(self.h, C.byref(req), C.byref(rid)))
        self.inflight[rid.value] = (q, qv, scratch, r, g, len(basis), want_gram, keep, req)
        return rid.value

    def step(self):
        n = max(len(self.inflight), 1)
        ids = (C.c_int64 * n)()
        sts = (C.c_int * n)()
        nd = C.c_int32(0)
        self.ctx.call_with_ws(lambda: self.ctx.lib.tt_engine_step(self.h, n, ids, sts, C.byref(nd)))
        out = {}
        for k in range(nd.value):
            q, qv, scratch, r, g, b, want_gram, keep, req = self.inflight.pop(ids[k])
            if sts[k] == 0:
                q.r = [int(qv.r[i]) for i in range(q.d + 1)]
                q.data = _packed(q.data, q.size())
            out[ids[k]] = (_STATUS.get(sts[k], sts[k]), q, np.array(r[: b + 1]),
                           np.array(g[:b]) if want_gram else None)
        return out

    def pending(self):
        return int(self.ctx.lib.tt_engine_pending(self.h))
