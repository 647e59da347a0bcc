"""Planted mistakes in copies of oracle routines must be caught by the pins.

Each mutant is a plausible slip (a transposed operand, a misplaced
coefficient, a wrong threshold, a strict instead of non-strict test); the
same independent reference used by the pins has to reject it.  The real
oracle is never modified.
"""
import math

import numpy as np

import oracle
from oracle import tt_full
from paper_2211_08770_amd import synth


def _dot_transposed(x, y):
    W = np.ones((1, 1))
    for X, Y in zip(x, y):
        Wn = np.zeros((X.shape[2], Y.shape[2]))
        for i in range(X.shape[1]):
            Wn += X[:, i, :].T @ W @ Y[:, i, :][:, ::-1]      # slip: reversed column order
        W = Wn
    return float(W[0, 0])


def _sum_coef_everywhere(terms):
    return oracle.tt_sum([(1.0, [c * a for c in x]) for a, x in terms])   # slip: coef on every core


def _select_rank_strict(sigma, eps, max_rank=None):
    s = np.asarray(sigma)
    for t in range(1, s.size + 1):
        if math.sqrt(np.sum(s[t:] ** 2)) < eps:                # slip: strict inequality
            return t, 1.0
    return s.size, 1.0


def _round_wrong_threshold(cores, delta):
    d = len(cores)
    return oracle.tt_round(cores, delta * math.sqrt(d - 1) / math.sqrt(d))   # slip: sqrt(d)


def test_dense_dot_pin_catches_transposed_operand():
    g = synth.rng(60)
    x = synth.random_tt(g, [3, 4, 3], [1, 2, 3, 1])
    y = synth.random_tt(g, [3, 4, 3], [1, 2, 3, 1])
    ref = float(np.vdot(tt_full(x).ravel(), tt_full(y).ravel()))
    assert abs(oracle.tt_dot(x, y) - ref) < 1e-12 * (abs(ref) + 1)
    assert abs(_dot_transposed(x, y) - ref) > 1e-6 * (abs(ref) + 1)


def test_dense_sum_pin_catches_misplaced_coefficient():
    g = synth.rng(61)
    terms = [(2.0, synth.random_tt(g, [3, 3, 3], [1, 2, 2, 1])), (-0.5, synth.random_tt(g, [3, 3, 3], [1, 2, 2, 1]))]
    ref = sum(a * tt_full(x) for a, x in terms)
    assert np.allclose(tt_full(oracle.tt_sum(terms)), ref, atol=1e-12)
    assert not np.allclose(tt_full(_sum_coef_everywhere(terms)), ref, atol=1e-6)


def test_tie_pin_catches_strict_inequality():
    s = np.array([4.0, 3.0, 2.0, 1.0])
    assert oracle.select_rank(s, 1.0)[0] == 3
    assert _select_rank_strict(s, 1.0)[0] != 3


def test_eckart_young_pin_catches_wrong_threshold():
    # d = 2 with a tail between delta/sqrt(2)*||X|| and delta*||X||.
    g = synth.rng(62)
    U, _ = np.linalg.qr(g.standard_normal((6, 4)))
    V, _ = np.linalg.qr(g.standard_normal((5, 4)))
    sig = np.array([1.0, 0.5, 0.08, 0.0])
    X = (U * sig) @ V.T
    nx = np.linalg.norm(X)
    delta = 0.1 / nx                       # tail after rank 2 is 0.08 = 0.8 * delta * ||X||
    x = [X.reshape(1, 6, 5), np.eye(5).reshape(5, 5, 1)]
    best = (U[:, :2] * sig[:2]) @ V[:, :2].T
    assert np.allclose(tt_full(oracle.tt_round(x, delta)), best, atol=1e-13)
    assert not np.allclose(tt_full(_round_wrong_threshold(x, delta)), best, atol=1e-6)
