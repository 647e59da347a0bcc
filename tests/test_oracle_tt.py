"""Pins of the oracle's TT primitives against dense brute force, closed forms and invariants.

Nothing here re-derives a result with the oracle's own formula: each check
compares the oracle to an independent computation (dense NumPy/LAPACK on the
full tensor, a closed form, or a structural invariant of the paper's
Section 2).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import tt_full, tt_dot, tt_axpy, tt_sum, tt_round, tt_ranks, RoundLog
from paper_2211_08770_amd import synth


def rand_tt(seed, ns, ranks, scale=1.0):
    return synth.random_tt(synth.rng(seed), ns, ranks, np.float64, scale)


SHAPES = [
    ([5], [1, 1]),
    ([3, 4], [1, 3, 1]),
    ([4, 3, 5], [1, 2, 3, 1]),
    ([2, 3, 2, 3], [1, 2, 4, 3, 1]),
    ([3, 3, 3, 3, 3], [1, 3, 5, 5, 2, 1]),
]


@pytest.mark.parametrize("ns,ranks", SHAPES)
def test_full_entries_are_slice_products(ns, ranks):
    # Section 2: x(i_1..i_d) = X_1(i_1) X_2(i_2) ... X_d(i_d), entry by entry.
    x = rand_tt(1, ns, ranks)
    F = tt_full(x)
    for idx in np.ndindex(*ns):
        m = np.eye(1)
        for k, i in enumerate(idx):
            m = m @ x[k][:, i, :]
        assert abs(F[idx] - m[0, 0]) <= 1e-12 * (1 + abs(m[0, 0]))


def test_full_rank1_is_outer_product():
    g = synth.rng(2)
    vs = [g.standard_normal(n) for n in (3, 4, 2, 5)]
    cores = [v.reshape(1, -1, 1) for v in vs]
    ref = np.einsum("a,b,c,d->abcd", *vs)
    assert np.allclose(tt_full(cores), ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("ns,ranks", SHAPES)
def test_dot_matches_dense(ns, ranks):
    x = rand_tt(3, ns, ranks)
    y = rand_tt(4, ns, [1] + [max(1, r - 1) for r in ranks[1:-1]] + [1])
    ref = float(np.vdot(tt_full(x).ravel(), tt_full(y).ravel()))
    got = tt_dot(x, y)
    scale = np.linalg.norm(tt_full(x)) * np.linalg.norm(tt_full(y))
    assert abs(got - ref) <= 1e-13 * scale


def test_dot_rank1_closed_form():
    # <u_1 o ... o u_d, v_1 o ... o v_d> = prod_k <u_k, v_k>
    g = synth.rng(5)
    us = [g.standard_normal(n) for n in (4, 3, 6)]
    vs = [g.standard_normal(n) for n in (4, 3, 6)]
    x = [u.reshape(1, -1, 1) for u in us]
    y = [v.reshape(1, -1, 1) for v in vs]
    ref = math.prod(float(u @ v) for u, v in zip(us, vs))
    assert abs(tt_dot(x, y) - ref) <= 1e-14 * math.prod(np.linalg.norm(u) * np.linalg.norm(v) for u, v in zip(us, vs))


def test_dot_is_symmetric_and_bilinear():
    ns = [3, 4, 3]
    x = rand_tt(6, ns, [1, 2, 3, 1])
    y = rand_tt(7, ns, [1, 3, 2, 1])
    z = rand_tt(8, ns, [1, 2, 2, 1])
    assert abs(tt_dot(x, y) - tt_dot(y, x)) <= 1e-12 * abs(tt_dot(x, y))
    lhs = tt_dot(tt_axpy(2.5, x, y), z)
    rhs = 2.5 * tt_dot(x, z) + tt_dot(y, z)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("ns,ranks", SHAPES)
def test_axpy_matches_dense_and_ranks_add(ns, ranks):
    x = rand_tt(9, ns, ranks)
    yr = [1] + [r + 1 for r in ranks[1:-1]] + [1]
    y = rand_tt(10, ns, yr)
    z = tt_axpy(-0.75, x, y)
    assert np.allclose(tt_full(z), -0.75 * tt_full(x) + tt_full(y), rtol=0, atol=1e-12)
    if len(ns) > 1:
        # Section 2: the k-th TT-rank of a sum is r_k + s_k.
        assert tt_ranks(z)[1:-1] == [a + b for a, b in zip(ranks[1:-1], yr[1:-1])]


def test_lazy_sum_matches_dense():
    ns = [3, 2, 4, 3]
    terms = [(c, rand_tt(20 + i, ns, [1, 2, 3, 2, 1])) for i, c in enumerate((1.0, -2.0, 0.5, 3.0))]
    ref = sum(c * tt_full(x) for c, x in terms)
    assert np.allclose(tt_full(tt_sum(terms)), ref, rtol=0, atol=1e-12)


def test_norm_after_right_to_left_sweep():
    # After the R-to-L sweep the cores 2..d are right-orthonormal, so ||x|| = ||G_1||_F.
    x = rand_tt(11, [4, 3, 5, 2], [1, 3, 4, 2, 1])
    G, _ = oracle.tt_orth_rl(x)
    assert abs(np.linalg.norm(G[0]) - np.linalg.norm(tt_full(x))) <= 1e-13 * np.linalg.norm(tt_full(x))
    for k in range(1, len(G)):
        r0, n, r1 = G[k].shape
        M = G[k].reshape(r0, n * r1)
        assert np.allclose(M @ M.T, np.eye(r0), atol=1e-13)


def test_select_rank_cases():
    s = np.array([4.0, 3.0, 2.0, 1.0])
    # tails: t=1 -> sqrt(14), t=2 -> sqrt(5), t=3 -> 1, t=4 -> 0
    assert oracle.select_rank(s, 1.0)[0] == 3          # tail exactly eps is accepted
    assert oracle.select_rank(s, 0.999)[0] == 4
    assert oracle.select_rank(s, math.sqrt(5))[0] == 2
    assert oracle.select_rank(s, 100.0)[0] == 1        # rank never drops below 1
    assert oracle.select_rank(s, 0.0)[0] == 4
    assert oracle.select_rank(s, 0.0, max_rank=2)[0] == 2
    assert oracle.select_rank(np.array([2.0, 0.0, 0.0]), 0.0)[0] == 1


@pytest.mark.parametrize("delta", [1e-1, 1e-3, 1e-8])
def test_round_d2_is_eckart_young(delta):
    # d = 2: eps = delta * ||X|| and TT-round is the truncated SVD of the matrix.
    g = synth.rng(12)
    U, _ = np.linalg.qr(g.standard_normal((9, 7)))
    V, _ = np.linalg.qr(g.standard_normal((8, 7)))
    sig = 10.0 ** (-np.arange(7) * 1.3)
    X = (U * sig) @ V.T
    x = [X.reshape(1, 9, 8), np.eye(8).reshape(8, 8, 1)]
    xr = tt_round(x, delta)
    nx = np.linalg.norm(X)
    t = next(t for t in range(1, 8) if math.sqrt(np.sum(sig[t:] ** 2)) <= delta * nx)
    best = (U[:, :t] * sig[:t]) @ V[:, :t].T
    assert tt_ranks(xr) == [1, t, 1]
    assert np.allclose(tt_full(xr), best, rtol=0, atol=1e-13 * nx)


@pytest.mark.parametrize("cap", [1, 2, 4])
def test_round_d2_rank_cap_is_the_best_rank_k_approximation(cap):
    # d = 2 with delta = 0 and a rank cap k: the truncated SVD at rank k (Eckart-Young), the
    # rank-capped rounding the paper applies to its Krylov inputs with k = 1 (Section 4)
    g = synth.rng(13)
    X = g.standard_normal((9, 4)) @ g.standard_normal((4, 8)) + 1e-3 * g.standard_normal((9, 8))
    U, sig, Vt = np.linalg.svd(X, full_matrices=False)
    x = [X.reshape(1, 9, 8), np.eye(8).reshape(8, 8, 1)]
    xr = tt_round(x, 0.0, max_rank=cap)
    best = (U[:, :cap] * sig[:cap]) @ Vt[:cap]
    assert tt_ranks(xr) == [1, cap, 1]
    assert np.allclose(tt_full(xr), best, rtol=0, atol=1e-13 * np.linalg.norm(X))


def _rand_sum(seed, ns, comp_rank, ncomp, decay=0.3):
    terms = []
    d = len(ns)
    for c in range(ncomp):
        ranks = [1] + [comp_rank] * (d - 1) + [1]
        terms.append((decay ** c, rand_tt(seed + 100 * c, ns, ranks)))
    return terms


ROUND_CASES = [
    ([6, 5, 4], 3, 4),
    ([4, 4, 4, 4], 2, 5),
    ([3, 5, 3, 4, 3], 2, 3),
    ([8, 8], 4, 3),
]


@pytest.mark.parametrize("ns,cr,nc", ROUND_CASES)
@pytest.mark.parametrize("delta", [1e-2, 1e-5, 1e-10])
def test_round_error_bound_ranks_and_orthonormality(ns, cr, nc, delta):
    x = tt_sum(_rand_sum(13, ns, cr, nc))
    F = tt_full(x)
    nx = np.linalg.norm(F)
    lg = RoundLog()
    xr = tt_round(x, delta, log=lg)
    # Section 2: ||x - x~|| <= delta ||x||
    err = np.linalg.norm(F - tt_full(xr))
    assert err <= delta * nx * (1 + 1e-10) + 1e-14 * nx
    # ranks never exceed the input ranks nor the bond caps
    caps = oracle.tt_rank_caps(ns)
    for a, b, c in zip(tt_ranks(xr), tt_ranks(x), caps):
        assert a <= b and a <= c
    # cores 1..d-1 are left-orthonormal; ||x~|| = ||G_d||_F
    for k in range(len(xr) - 1):
        r0, n, r1 = xr[k].shape
        L = xr[k].reshape(r0 * n, r1)
        assert np.allclose(L.T @ L, np.eye(r1), atol=1e-13)
    assert abs(np.linalg.norm(xr[-1]) - np.linalg.norm(tt_full(xr))) <= 1e-12 * nx
    assert abs(np.linalg.norm(tt_full(xr)) - nx) <= delta * nx * (1 + 1e-10)
    assert abs(lg.norm - nx) <= 1e-13 * nx


@pytest.mark.parametrize("ns,cr,nc", ROUND_CASES)
@pytest.mark.parametrize("delta", [1e-2, 1e-6])
def test_round_matches_dense_tt_svd(ns, cr, nc, delta):
    # The two-sweep rounding sees the same per-bond spectra as the dense TT-SVD
    # of the full tensor with the same absolute threshold.
    x = tt_sum(_rand_sum(14, ns, cr, nc))
    F = tt_full(x)
    nx = np.linalg.norm(F)
    eps = delta / math.sqrt(len(ns) - 1) * nx
    ref, ref_sig = oracle.tt_svd(F, eps)
    lg = RoundLog()
    xr = tt_round(x, delta, log=lg)
    assert tt_ranks(xr) == tt_ranks(ref)
    for s_tt, s_dense in zip(lg.sigmas, ref_sig):
        k = min(len(s_tt), len(s_dense))
        assert np.allclose(s_tt[:k], s_dense[:k], rtol=0, atol=1e-12 * nx)
        assert np.all(np.abs(s_tt[k:]) <= 1e-12 * nx) and np.all(np.abs(s_dense[k:]) <= 1e-12 * nx)
    assert np.allclose(tt_full(xr), tt_full(ref), rtol=0, atol=1e-11 * nx)


def test_round_identity_on_exact_low_rank():
    # A TT with minimal ranks and every bond singular value far above eps is
    # returned unchanged (same ranks, same tensor).
    ns = [5, 6, 5, 4]
    x = rand_tt(15, ns, [1, 3, 4, 3, 1])
    F = tt_full(x)
    lg = RoundLog()
    xr = tt_round(x, 1e-9, log=lg)
    assert all(s[s > 1e-12 * lg.norm].min() > 1e3 * lg.eps for s in lg.sigmas)
    assert tt_ranks(xr) == tt_ranks(x)
    assert np.allclose(tt_full(xr), F, rtol=0, atol=1e-13 * np.linalg.norm(F))


def test_round_compresses_duplicated_sum_back():
    # x + x has ranks 2r but exact ranks r: rounding recovers r and 2x.
    ns = [4, 5, 4]
    x = rand_tt(16, ns, [1, 3, 2, 1])
    s = tt_sum([(1.0, x), (1.0, x)])
    xr = tt_round(s, 1e-10)
    assert tt_ranks(xr) == [1, 3, 2, 1]
    assert np.allclose(tt_full(xr), 2 * tt_full(x), atol=1e-12 * np.linalg.norm(tt_full(x)))


def test_round_special_cases():
    # d = 1: a copy
    x1 = rand_tt(17, [7], [1, 1])
    assert np.array_equal(tt_round(x1, 0.5)[0], x1[0])
    # zero tensor: rank-1 zeros
    z = [np.zeros((1, 3, 2)), np.zeros((2, 4, 2)), np.zeros((2, 3, 1))]
    zr = tt_round(z, 1e-3)
    assert tt_ranks(zr) == [1, 1, 1, 1] and all(not c.any() for c in zr)
    # delta = 0 reproduces the tensor
    x = tt_sum(_rand_sum(18, [3, 4, 3], 2, 3))
    xr = tt_round(x, 0.0)
    assert np.allclose(tt_full(xr), tt_full(x), atol=1e-13 * np.linalg.norm(tt_full(x)))
    # max_rank caps every bond
    xr1 = tt_round(x, 0.0, max_rank=1)
    assert tt_ranks(xr1) == [1, 1, 1, 1]
    with pytest.raises(ValueError):
        tt_round(x, -1.0)


def test_compression_measures():
    ns = [4, 5, 6]
    x = rand_tt(19, ns, [1, 2, 3, 1])
    assert oracle.compression_ratio(x) == (1 * 4 * 2 + 2 * 5 * 3 + 3 * 6 * 1) / (4 * 5 * 6)
    s = tt_sum([(1.0, x), (1.0, x)])
    xr = tt_round(s, 1e-10)
    assert oracle.compression_gain(s, xr) == pytest.approx(
        (4 * 4 + 4 * 5 * 6 + 6 * 6) / (1 * 4 * 2 + 2 * 5 * 3 + 3 * 6 * 1))
