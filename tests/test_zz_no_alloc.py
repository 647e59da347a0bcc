"""tt_dot_noalloc (the allocation-free variant of tt_dot, for callers that cannot
allocate) called through the C ABI against tt_dot on the same pairs: two calls
in a row, the second with a smaller pair, in both dtypes, plus its argument
and capacity errors (returned before any launch)."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from paper_2211_08770_amd import synth
from gpu_util import need_gpu, dev_tt

pytestmark = pytest.mark.gpu


def _lib():
    tt = need_gpu()
    lib = tt._load()
    lib.tt_dot_noalloc.argtypes = [C.c_void_p, C.POINTER(tt._Vec), C.POINTER(tt._Vec), C.c_void_p]
    lib.tt_dot_noalloc.restype = C.c_int
    return tt, lib


def _noalloc_dot(lib, x, y, out):
    vx, vy = x._vec(), y._vec()
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.tt_dot_noalloc(C.c_void_p(stream), C.byref(vx), C.byref(vy), C.c_void_p(out.data_ptr()))
    return st


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_dot_matches_tt_dot_twice_second_smaller(dtype):
    tt, lib = _lib()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    g = synth.rng(90)
    big = ([12, 40, 9, 33], [1, 24, 37, 18, 1], [1, 30, 5, 41, 1])
    small = ([3, 5, 4], [1, 2, 3, 1], [1, 4, 1, 1])
    out = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
    for call, (ns, rx, ry) in enumerate((big, small)):
        x = [c.astype(npdt) for c in synth.random_tt(g, ns, rx)]
        y = [c.astype(npdt) for c in synth.random_tt(g, ns, ry)]
        X, Y = dev_tt(x, dtype), dev_tt(y, dtype)
        want = tt.dot(X, Y)
        assert _noalloc_dot(lib, X, Y, out[call:]) == 0
        torch.cuda.synchronize()
        got = float(out[call].item())
        up = lambda v: [c.astype(np.float64) for c in v]
        scale = oracle.tt_norm(up(x)) * oracle.tt_norm(up(y))
        # same contraction, same order of operations as tt_dot: equal to its result
        assert abs(got - want) <= 1e-14 * scale, (call, got, want)
        assert abs(got - oracle.tt_dot(up(x), up(y))) <= 1e-12 * scale


def test_noalloc_dot_errors_before_launch():
    tt, lib = _lib()
    g = synth.rng(91)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    x = dev_tt(synth.random_tt(g, [4, 5], [1, 3, 1]))
    y = dev_tt(synth.random_tt(g, [4, 6], [1, 3, 1]))
    assert _noalloc_dot(lib, x, y, out) == -1          # mode sizes differ: TT_EINVAL
    # a pair whose intermediate needs more than the 16 MiB scratch: TT_ECAPACITY
    big = tt.TT(torch.zeros(1, dtype=torch.float64, device="cuda"), [4096, 2], [1, 1024, 1])
    vb = big._vec()
    vb.capacity = 4096 * 1024 * 2     # claims the packed size; nothing is read before the check
    st = lib.tt_dot_noalloc(C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(vb), C.byref(vb),
                            C.c_void_p(out.data_ptr()))
    assert st == -3
    torch.cuda.synchronize()
