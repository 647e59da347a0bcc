"""Pins of the oracle's Laplacian TT-matrix and Krylov inputs (Section 4).

Independent references: the closed-form eigenpairs of the Dirichlet second
difference, the dense Kronecker sum applied axis by axis to the full tensor,
and, for the Krylov recipe, the dense power sequence (order 1, where rank one
is exact) and the best rank-one approximation by a dense SVD (order 2, where
TT-rounding to rank one is Eckart-Young).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import tt_full
from paper_2211_08770_amd import synth


def dense_laplacian_apply(T):
    out = np.zeros_like(T)
    for k, n in enumerate(T.shape):
        L = oracle.laplacian_1d(n)
        out += np.moveaxis(np.tensordot(L, T, axes=(1, k)), 0, k)
    return out


def test_laplacian_1d_eigenpairs():
    for n in (1, 2, 5, 15):
        L = oracle.laplacian_1d(n)
        h = 1.0 / (n + 1)
        for k in range(1, n + 1):
            v = np.sin(np.pi * k * np.arange(1, n + 1) / (n + 1))
            lam = -4.0 / h ** 2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2
            assert np.allclose(L @ v, lam * v, rtol=0, atol=1e-9 * abs(lam))


@pytest.mark.parametrize("ns,ranks", [([6], [1, 1]), ([4, 5], [1, 3, 1]), ([3, 4, 5], [1, 2, 3, 1]),
                                      ([2, 3, 2, 4], [1, 2, 2, 3, 1]), ([1, 3, 2], [1, 1, 2, 1])])
def test_tt_laplacian_matches_dense_kronecker_sum(ns, ranks):
    g = synth.rng(80)
    x = synth.random_tt(g, ns, ranks)
    y = oracle.tt_laplacian(x, -0.75)
    d = len(ns)
    assert oracle.tt_ranks(y) == ([1] + [2 * r for r in ranks[1:-1]] + [1] if d > 1 else [1, 1])
    ref = -0.75 * dense_laplacian_apply(tt_full(x))
    assert np.allclose(tt_full(y), ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_tt_laplacian_on_eigen_tensor():
    ns = [4, 6, 5]
    ks = [2, 1, 4]
    cores, lam = [], 0.0
    for n, k in zip(ns, ks):
        v = np.sin(np.pi * k * np.arange(1, n + 1) / (n + 1))
        cores.append(v.reshape(1, n, 1))
        lam += -4.0 * (n + 1) ** 2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2
    y = oracle.tt_laplacian(cores)
    assert np.allclose(tt_full(y), lam * tt_full(cores), rtol=0, atol=1e-9 * abs(lam))


def test_krylov_order_one_is_the_normalised_power_sequence():
    n, m = 7, 6
    A = oracle.krylov_inputs([n], m)
    L = oracle.laplacian_1d(n)
    v = np.ones(n)
    for j in range(m):
        w = v / np.linalg.norm(v)
        assert np.allclose(tt_full(A[j]), w, rtol=0, atol=1e-12)
        v = -L @ w


def test_krylov_order_two_is_the_best_rank_one_sequence():
    ns, m = [5, 4], 6
    A = oracle.krylov_inputs(ns, m)
    X = np.ones(ns)
    for j in range(m):
        U, S, Vt = np.linalg.svd(X)
        best = np.outer(U[:, 0], Vt[0])           # normalised best rank-one approximation
        assert np.allclose(tt_full(A[j]), best, rtol=0, atol=1e-11)
        X = -dense_laplacian_apply(best)


def test_krylov_inputs_are_unit_rank_one_and_increasingly_ill_conditioned():
    A = oracle.krylov_inputs([15, 15, 15], 20)
    kappa = []
    cols = []
    for a in A:
        assert oracle.tt_ranks(a) == [1, 1, 1, 1]
        assert abs(oracle.tt_norm(a) - 1.0) < 1e-13
        cols.append(tt_full(a).ravel())
        kappa.append(np.linalg.cond(np.stack(cols, axis=1)))
    assert all(b >= a * (1 - 1e-9) for a, b in zip(kappa, kappa[1:]))
    assert kappa[-1] > 1e6
