"""Host planning of column-blocked QR: TT-sums whose unfoldings have more than 800 rows
and more than 400 columns are planned (in column blocks of 384) instead of rejected, the
workspace grows with the summed rank, and the SVD limit applies where ranks are planned
at their bounds.  Descriptors only: the data pointers are never dereferenced, no GPU."""
import ctypes as C

import pytest

from paper_2211_08770_amd import tt


def host_sum(ns, r, ncomp, dtype=0):
    d = len(ns)
    ranks = [1] + [r] * (d - 1) + [1]
    vecs = (tt._Vec * ncomp)()
    for v in vecs:
        v.d, v.dtype = d, dtype
        for k in range(d):
            v.n[k] = ns[k]
        for k in range(d + 1):
            v.r[k] = ranks[k]
        v.data = 4096   # never read by the planner
        v.capacity = sum(ranks[k] * ns[k] * ranks[k + 1] for k in range(d))
    coef = (C.c_double * ncomp)(*[1.0] * ncomp)
    return tt._Sum(ncomp, coef, vecs), (vecs, coef)


def ws_bytes(ns, r, ncomp, dtype=0):
    s, keep = host_sum(ns, r, ncomp, dtype)
    return tt._load().tt_round_workspace_bytes(C.byref(s))


@pytest.mark.parametrize("dtype", [0, 1])
def test_wide_unfoldings_are_planned(dtype):
    # 1024 x 400 fits one tree; 1024 x 500 and 16000 x 500 (50 terms of rank 10, n = 32) and
    # 4096 x 1024, 65536 x 1024 (64 terms of rank 16, n = 64) need column blocks
    a = ws_bytes([32] * 4, 10, 40, dtype)
    b = ws_bytes([32] * 4, 10, 50, dtype)
    c = ws_bytes([64] * 4, 16, 64, dtype)
    assert 0 < a < b < c


def test_blocked_workspace_grows_with_rank():
    sizes = [ws_bytes([15] * 6, 20, nc) for nc in (20, 30, 45, 60)]
    assert all(s > 0 for s in sizes)
    assert sizes == sorted(sizes)


def test_fp32_bulk_needs_less_workspace():
    assert 0 < ws_bytes([32] * 4, 10, 50, 1) < ws_bytes([32] * 4, 10, 50, 0)


def test_column_blocks_keep_only_factored_columns():
    # 100 components of rank 20 on order 6, n = 15: right-to-left unfoldings up to 30000 x 2000
    # in FP64.  Full-width tiles for every column block would take about M N^2 / 384 elements
    # per tree (about 10 GiB for the 30000 x 2000 one alone); with the blocks sharing one
    # full-width region and keeping only their factored columns the whole rounding's workspace
    # stays below 12 GiB.
    assert 0 < ws_bytes([15] * 6, 20, 100) < 12 * 2**30


def test_wide_svd_limit_applies_at_planning_time_only_for_bounds():
    # The left-to-right R factors of this sum have up to 2000 rows (above the 1024-row
    # one-workgroup kernel, below the 4096 of the block Jacobi): host planning accepts it
    assert ws_bytes([15] * 6, 20, 100) > 0
