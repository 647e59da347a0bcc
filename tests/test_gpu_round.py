"""GPU TT-round (through the C ABI) against the FP64 oracle.

Results are compared by reconstruction: the norm of the TT difference between
the GPU and oracle roundings, relative to ||x||, must be <= 1e-12 in FP64 and
<= max(delta, 1e-5) in FP32-bulk (the oracle runs on the FP32 input values
upcast exactly).  Ranks must match unless the oracle's truncation decision
sits within rounding of a tie (margin < 1 + 1e-8 in FP64, 1 + 1e-3 in FP32);
then only the error bound and the mutual distance are checked.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2211_08770_amd import synth
from gpu_util import need_gpu, dev_sum, host_cores, diff_norm, left_orth_error, sample_entries, rand_index, min_margin

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: None}
TIE = {torch.float64: 1 + 1e-8, torch.float32: 1 + 1e-3}


def rand_terms(seed, ns, ranks_list, coefs=None, scales=None):
    g = synth.rng(seed)
    terms = []
    for i, rk in enumerate(ranks_list):
        sc = 1.0 if scales is None else scales[i]
        terms.append((1.0 if coefs is None else coefs[i], synth.random_tt(g, ns, rk, np.float64, sc)))
    return terms


def check_round(terms, delta, dtype, max_rank=0, tol=None):
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    terms = [(a, [c.astype(npdt) for c in x]) for a, x in terms]
    x = oracle.tt_sum([(a, [c.astype(np.float64) for c in x]) for a, x in terms])
    lg = oracle.RoundLog()
    ref = oracle.tt_round(x, delta, max_rank=max_rank or None, log=lg)
    nx = lg.norm
    out, nrm = tt.round(dev_sum(terms, dtype), delta, max_rank=max_rank, return_norm=True)
    got = host_cores(out)
    if tol is None:
        tol = TOL[dtype] if dtype == torch.float64 else max(delta, 1e-5)
    assert abs(nrm - nx) <= max(tol, 1e-13) * max(nx, 1e-300) + (0 if nx else 1e-300)
    if nx == 0.0:
        # the zero tensor comes back with all ranks 1; its cores 1..d-1 are unit
        # vectors (left-orthonormal) and the last core is zero
        assert out.r == [1] * (len(x) + 1)
        assert not np.any(got[-1])
        assert left_orth_error(got) <= 1e-15
        return out
    d = diff_norm(got, ref) / nx
    de = tt.effective_delta(dev_sum(terms, dtype), delta)
    if de > delta:
        # FP32-bulk below its resolution: the per-bond threshold is the FP32 floor, so the
        # result meets delta_eff (not delta) and stays within delta_eff + delta of the oracle's
        err = diff_norm(got, x) / nx
        assert err <= de, (err, de)
        assert d <= de + delta, (d, de)
        assert all(a <= b for a, b in zip(out.r, oracle.tt_ranks(ref)))
        return out
    if min_margin(lg) >= TIE[dtype]:
        assert out.r == oracle.tt_ranks(ref), (out.r, oracle.tt_ranks(ref))
        assert d <= tol, d
    else:
        err = diff_norm(got, x) / nx
        assert err <= delta * (1 + 1e-10) + tol
        assert d <= 2 * delta + tol
    if dtype == torch.float64:
        assert left_orth_error(got) <= 1e-12
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("delta", [1e-1, 1e-4, 1e-10])
def test_round_small_sums(dtype, delta):
    ns = [5, 6, 4, 7]
    terms = rand_terms(100, ns, [[1, 3, 4, 2, 1], [1, 2, 2, 2, 1], [1, 4, 3, 3, 1]], coefs=[1.0, -0.5, 0.25],
                       scales=[1.0, 0.3, 0.01])
    check_round(terms, delta, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_round_orders_one_to_six(dtype):
    for d in range(1, 7):
        ns = [3 + (k % 3) for k in range(d)]
        rk = [1] + [2 + (k % 2) for k in range(d - 1)] + [1]
        terms = rand_terms(200 + d, ns, [rk, rk], coefs=[1.0, 2.0])
        check_round(terms, 1e-3, dtype)


def test_round_wide_and_tall_unfoldings():
    # first bond capped by n_1 = 2 (wide right-to-left QR), large middle ranks
    terms = rand_terms(300, [2, 9, 9, 3], [[1, 2, 12, 3, 1]] * 3)
    check_round(terms, 1e-6, torch.float64)


def test_round_multi_leaf_tsqr():
    # (n * s) = 64 * 30 = 1920 rows > one tile: several TSQR leaves and a tree
    terms = rand_terms(310, [8, 64, 64, 8], [[1, 8, 30, 8, 1]] * 2, scales=[1.0, 0.1])
    check_round(terms, 1e-8, torch.float64)
    check_round(terms, 1e-4, torch.float32)


def test_round_zero_tensor_and_caps():
    zero = [(0.0, [np.ones((1, 3, 2)), np.ones((2, 4, 2)), np.ones((2, 3, 1))])]
    check_round(zero, 1e-3, torch.float64)
    terms = rand_terms(320, [4, 5, 4], [[1, 3, 3, 1]] * 2)
    out = check_round(terms, 0.0, torch.float64, max_rank=1)
    assert out.r == [1, 1, 1, 1]


def test_round_delta_zero_reproduces():
    terms = rand_terms(330, [3, 4, 3, 4], [[1, 2, 3, 2, 1]] * 2)
    check_round(terms, 0.0, torch.float64)


@pytest.mark.parametrize("delta", [1e-4, 1e-8])
def test_round_graded_sum_of_20_terms_fp64(delta):
    # 20 rank-10 TTs, d = 8, n = 32, term j scaled by 2^-j on every core: input rank 200
    terms = synth.sum_of_graded_terms()
    out = check_round(terms, delta, torch.float64)
    expect = {1e-4: 20, 1e-8: 40}[delta]
    assert max(out.r) == expect


def test_round_graded_sum_of_20_terms_fp32():
    terms = synth.sum_of_graded_terms(dtype=np.float32)
    out = check_round(terms, 1e-4, torch.float32)
    # sampled entries against the oracle, relative to the largest entry magnitude
    x = oracle.tt_sum([(a, [c.astype(np.float64) for c in t]) for a, t in terms])
    ref = oracle.tt_round(x, 1e-4)
    idx = rand_index([32] * 8, 200, seed=3)
    e_ref = sample_entries(ref, idx)
    e_got = sample_entries(host_cores(out), idx)
    assert np.max(np.abs(e_ref - e_got)) <= 1e-4 * np.max(np.abs(e_ref))


def test_round_graded_sum_of_20_terms_fp32_at_1e8():
    """FP32-bulk at delta = 1e-8, below its resolution: rounded at delta_eff (the FP32
    floor of the per-bond threshold), against the oracle's rounding at 1e-8."""
    tt = need_gpu()
    terms = synth.sum_of_graded_terms(dtype=np.float32)
    de = tt.effective_delta(dev_sum(terms, torch.float32), 1e-8)
    assert 1e-8 < de < 1e-5
    out = check_round(terms, 1e-8, torch.float32)
    assert 20 < max(out.r) <= 40


def test_round_is_deterministic():
    tt = need_gpu()
    terms = synth.sum_of_graded_terms(nterms=6, d=5, n=16, r=6)
    a = tt.round(dev_sum(terms), 1e-6)
    b = tt.round(dev_sum(terms), 1e-6)
    assert a.r == b.r and torch.equal(a.data, b.data)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_round_wide_paths_are_deterministic(dtype):
    # the 1024 x 500 and 16000 x 500 unfoldings of 50 rank-10 components take column-blocked
    # QR and the 500-row R factors the block Jacobi SVD (its sweep counters are atomics, its
    # pairs run in any order): every call gives the same bits all the same
    tt = need_gpu()
    terms = rand_terms(322, [32, 32, 32, 32], [[1, 10, 10, 10, 1]] * 50,
                       scales=[2.0 ** -(j % 7) for j in range(50)])
    x = dev_sum(terms, dtype)
    a = tt.round(x, 1e-6)
    b = tt.round(x, 1e-6)
    assert a.r == b.r and a.r[2] > 224 and torch.equal(a.data, b.data)


def test_round_maximum_order():
    # d = 64, the largest order the library takes: 63 dependent steps in each sweep
    terms = rand_terms(320, [2] * 64, [[1] + [2] * 63 + [1], [1] + [1] * 63 + [1]], coefs=[1.0, -0.5])
    check_round(terms, 1e-10, torch.float64)


def test_round_order_above_maximum_is_rejected():
    tt = need_gpu()
    from paper_2211_08770_amd.tt import TT
    x = TT(torch.ones(65 * 2, dtype=torch.float64, device="cuda"), [2] * 65, [1] * 66)
    with pytest.raises(Exception):
        tt.round(x, 1e-8)


def test_round_at_the_tile_limits():
    # 40 components of rank 10 on order 4, n = 32: the right-to-left unfoldings are 1024 x 400,
    # the most columns a tile tree takes above 800 rows (nodes of two stacked 400 x 400
    # triangles fill an 800-row tile)
    terms = rand_terms(321, [32, 32, 32, 32], [[1, 10, 10, 10, 1]] * 40,
                       scales=[2.0 ** -(j % 7) for j in range(40)])
    check_round(terms, 1e-6, torch.float64)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_round_column_blocked_unfoldings(dtype):
    # 50 components of rank 10 on order 4, n = 32: the right-to-left unfoldings are
    # 1024 x 500 and 16000 x 500 and the second left-to-right one 1024 x 500, all more
    # than 800 rows and 400 columns: QR in column blocks (384 columns, then 116)
    terms = rand_terms(322, [32, 32, 32, 32], [[1, 10, 10, 10, 1]] * 50,
                       scales=[2.0 ** -(j % 7) for j in range(50)])
    out = check_round(terms, 1e-6, dtype)
    assert out.r[1] == 32 and out.r[2] > 300   # the left-to-right step 1 factors 1024 x 500


def test_round_column_blocked_three_blocks():
    # 64 components of rank 16 on order 4, n = 64, near two base TTs (so the result has low
    # rank): the right-to-left unfoldings are 4096 x 1024 and 65536 x 1024, blocked three
    # times (384 + 384 + 256 columns)
    g = synth.rng(323)
    ns = [64, 64, 64, 64]
    base = [synth.random_tt(g, ns, [1, 16, 16, 16, 1]) for _ in range(2)]
    terms = []
    for j in range(64):
        x = [c.copy() for c in base[j % 2]]
        x[1] = x[1] + 1e-3 * g.standard_normal(x[1].shape)
        terms.append((float(g.standard_normal()), x))
    check_round(terms, 1e-6, torch.float64)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_round_large_r_factor_block_jacobi(dtype):
    # 80 components of rank 16 on order 4, n = 64, near two base TTs: the left-to-right
    # step 1 factors a 2048 x 1280 matrix, and its 1280 x 1280 R factor (more than 1024
    # rows) takes the block Jacobi SVD over many workgroups
    g = synth.rng(324)
    ns = [64, 64, 64, 64]
    base = [synth.random_tt(g, ns, [1, 16, 16, 16, 1]) for _ in range(2)]
    terms = []
    for j in range(80):
        x = [c.copy() for c in base[j % 2]]
        x[1] = x[1] + 1e-3 * g.standard_normal(x[1].shape)
        terms.append((float(g.standard_normal()), x))
    out = check_round(terms, 1e-6, dtype)
    assert out.r[1] == 32
