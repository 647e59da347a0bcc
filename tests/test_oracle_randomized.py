"""Pins of the oracle's randomized rounding (Randomize-then-Orthogonalize).

Independent references: exact recovery of a sum whose true TT-ranks are at
most the sketch ranks (dense comparison), the randomized range finder of
Halko, Martinsson and Tropp at order two (Q Q^T X with Q = orth(X Omega),
dense), and the accuracy of the rounded result against the deterministic
error bound on a graded sum.
"""
import numpy as np

import oracle
from oracle import tt_full
from paper_2211_08770_amd import synth


def test_exact_recovery_when_sketch_ranks_cover_the_true_ranks():
    g = synth.rng(90)
    ns = [4, 5, 3, 4]
    base = synth.random_tt(g, ns, [1, 2, 3, 2, 1])
    other = synth.random_tt(g, ns, [1, 1, 2, 1, 1])
    terms = [(0.5, base), (0.3, base), (-0.7, other), (0.2, base)]       # lazy ranks 3+1+... true ranks <= 3, 5, 3
    sketch = synth.random_tt(g, ns, [1, 5, 7, 5, 1])
    y = oracle.tt_round_rto(terms, sketch)
    ref = sum(a * tt_full(x) for a, x in terms)
    assert np.allclose(tt_full(y), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert oracle.tt_ranks(y) == [1, 4, 7, 5, 1]                           # min(l_k, p_{k-1} n_k)


def test_order_two_is_the_randomized_range_finder():
    g = synth.rng(91)
    ns = [9, 7]
    terms = [(1.0, synth.random_tt(g, ns, [1, 5, 1])), (0.4, synth.random_tt(g, ns, [1, 3, 1]))]
    sketch = synth.random_tt(g, ns, [1, 4, 1])
    X = sum(a * tt_full(x) for a, x in terms)
    Omega = sketch[1][:, :, 0].T                                           # n_2 x l
    Q, _ = np.linalg.qr(X @ Omega)
    y = oracle.tt_round_rto(terms, sketch)
    assert np.allclose(tt_full(y), Q @ (Q.T @ X), rtol=0, atol=1e-12)


def test_rounded_result_meets_the_error_bound_on_a_graded_sum():
    g = synth.rng(92)
    ns = [8, 8, 8, 8]
    terms = [(1.0, [c * 2.0 ** -j for c in synth.random_tt(g, ns, [1, 4, 4, 4, 1])]) for j in range(6)]
    x = oracle.tt_sum(terms)
    delta = 1e-4
    det = oracle.tt_round(x, delta)
    lk = [1] + [min(r + 8, 64) for r in oracle.tt_ranks(det)[1:-1]] + [1]
    sketch = synth.random_tt(g, ns, lk)
    y = oracle.tt_round_rto(terms, sketch, delta)
    err = np.linalg.norm(tt_full(y) - tt_full(x)) / np.linalg.norm(tt_full(x))
    assert err <= 2 * delta
    assert all(a <= b + 2 for a, b in zip(oracle.tt_ranks(y), oracle.tt_ranks(det)))


def test_order_one_returns_the_sum():
    g = synth.rng(93)
    terms = [(2.0, synth.random_tt(g, [6], [1, 1])), (-1.0, synth.random_tt(g, [6], [1, 1]))]
    y = oracle.tt_round_rto(terms, synth.random_tt(g, [6], [1, 1]))
    assert np.allclose(tt_full(y), sum(a * tt_full(x) for a, x in terms))
