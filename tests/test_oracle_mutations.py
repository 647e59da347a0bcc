"""Planted mistakes in copies of oracle routines must be caught by the pins.

Each mutant is a plausible slip (a transposed operand, a misplaced
coefficient, a wrong threshold, a strict instead of non-strict test, the
cancelling Householder sign, the wrong canonical index order, a Gram breakdown
rule at the square root of the round-off); the same
independent reference used by the pins has to reject it.  The oracle's files
are never modified: a mutant is a separate function, swapped in for one test
at most.
"""
import math

import numpy as np

import oracle
from oracle import tt_full
from inputs import conditioned_inputs
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


def _tth_vec_cancelling_sign(a, F, delta, res):
    # slip: the sign printed in the TTH-vec listing, r(i) = +s gamma
    i = len(F)
    r = np.zeros(i)
    s = 0.0
    terms = [(1.0, a)]
    for j in range(i - 1):
        r[j] = oracle.tt_dot(a, F[j])
        s = s + r[j] ** 2
        terms.append((-r[j], F[j]))
    w = oracle.tt_round(oracle.tt_sum(terms), delta)
    sign = 1.0 if oracle.tt_dot(a, F[i - 1]) > 0.0 else -1.0
    r[i - 1] = sign * math.sqrt(oracle.tt_dot(a, a) - s)
    w = oracle.tt_round(oracle.tt_sum([(1.0, w), (-r[i - 1], F[i - 1])]), delta)
    return oracle.tt_scale(1.0 / oracle.tt_norm(w), w), r


def _canonical_index_last_fastest(i, ns):
    rest = i - 1
    idx = []
    for n in reversed(ns):                                      # slip: last index fastest
        idx.append(rest % n + 1)
        rest //= n
    return tuple(reversed(idx))


def _householder_vs_lapack(monkeypatch, name, mutant):
    import oracle.schemes as sch
    g = synth.rng(63)
    ns = [3, 4, 2]
    X = [[(1.0, synth.random_tt(g, ns, [1, 2, 2, 1]))] for _ in range(4)]
    A = np.stack([tt_full(oracle.tt_sum(x)).ravel(order="F") for x in X], axis=1)
    _, Rd = np.linalg.qr(A)
    assert np.allclose(oracle.householder(X, 1e-14).R, Rd, atol=1e-10)
    monkeypatch.setattr(sch, name, mutant)
    return np.allclose(sch.householder(X, 1e-14).R, Rd, atol=1e-6)


def test_lapack_pin_catches_cancelling_householder_sign(monkeypatch):
    assert not _householder_vs_lapack(monkeypatch, "tth_vec", _tth_vec_cancelling_sign)


def test_lapack_pin_catches_reversed_canonical_order(monkeypatch):
    assert not _householder_vs_lapack(monkeypatch, "canonical_index", _canonical_index_last_fastest)


def _tt_laplacian_transposed_blocks(cores, alpha=1.0):
    # slip: interior cores [[X, L X], [0, X]] (the block of the Laplacian in the wrong corner)
    d = len(cores)
    X = [np.asarray(c, dtype=np.float64) for c in cores]
    out = []
    for k in range(d):
        r0, n, r1 = X[k].shape
        LX = oracle.apply_along_mode(oracle.laplacian_1d(n), X[k])
        if k == 0:
            Y = np.concatenate([LX, X[k]], axis=2) * alpha
        elif k == d - 1:
            Y = np.concatenate([X[k], LX], axis=0)
        else:
            Y = np.zeros((2 * r0, n, 2 * r1))
            Y[:r0, :, :r1] = X[k]
            Y[:r0, :, r1:] = LX
            Y[r0:, :, r1:] = X[k]
        out.append(Y)
    return out


def test_dense_kronecker_pin_catches_misplaced_laplacian_block():
    g = synth.rng(64)
    ns = [3, 4, 3]
    x = synth.random_tt(g, ns, [1, 2, 2, 1])
    T = tt_full(x)
    ref = np.zeros_like(T)
    for k, n in enumerate(ns):
        ref += np.moveaxis(np.tensordot(oracle.laplacian_1d(n), T, axes=(1, k)), 0, k)
    assert np.allclose(tt_full(oracle.tt_laplacian(x)), ref, atol=1e-9 * np.abs(ref).max())
    assert not np.allclose(tt_full(_tt_laplacian_transposed_blocks(x)), ref, atol=1e-3 * np.abs(ref).max())


def _rto_wrong_sketch_core(terms, sketch, delta=0.0):
    # slip: the contraction for bond k uses sketch core k - 1 (off by one) where shapes allow
    sk = [sketch[0], sketch[0].reshape(sketch[1].shape) if sketch[0].size == sketch[1].size else sketch[1]]
    return oracle.tt_round_rto(terms, sk, delta)


def test_range_finder_pin_catches_a_wrong_sketch():
    g = synth.rng(65)
    ns = [6, 6]
    terms = [(1.0, synth.random_tt(g, ns, [1, 4, 1])), (0.5, synth.random_tt(g, ns, [1, 3, 1]))]
    sketch = synth.random_tt(g, ns, [1, 3, 1])
    X = sum(a * tt_full(x) for a, x in terms)
    Omega = sketch[1][:, :, 0].T
    Q, _ = np.linalg.qr(X @ Omega)
    assert np.allclose(tt_full(oracle.tt_round_rto(terms, sketch)), Q @ (Q.T @ X), atol=1e-12)
    bad = _rto_wrong_sketch_core(terms, sketch)
    assert not np.allclose(tt_full(bad), Q @ (Q.T @ X), atol=1e-6)


def _krylov_without_minus(ns, m):
    # slip: x_{j+1} = +Delta_d a_j
    x = oracle.tt_ones(ns)
    A = []
    for j in range(m):
        a = oracle.tt_round(x, 0.0, max_rank=1)
        a = oracle.tt_scale(1.0 / oracle.tt_norm(a), a)
        A.append(a)
        x = oracle.tt_laplacian(a, 1.0)
    return A


def test_power_sequence_pin_catches_the_missing_minus_sign():
    n, m = 7, 4
    L = oracle.laplacian_1d(n)
    v, ref = np.ones(n), []
    for _ in range(m):
        w = v / np.linalg.norm(v)
        ref.append(w)
        v = -L @ w
    good = oracle.krylov_inputs([n], m)
    bad = _krylov_without_minus([n], m)
    assert all(np.allclose(tt_full(a), r, atol=1e-12) for a, r in zip(good, ref))
    assert not all(np.allclose(tt_full(a), r, atol=1e-6) for a, r in zip(bad, ref))


def _gram_sqrt_u_rule(A):
    """The factorisation step of TT-Gram with the breakdown rule at sqrt(u) G_jj."""
    G = oracle.gram_of([oracle.tt_sum(a) for a in A])
    L = np.linalg.cholesky(G)
    u = np.finfo(np.float64).eps / 2
    if np.any(np.diag(L) ** 2 <= math.sqrt(u) * np.diag(G)):          # slip: sqrt(u) for m u
        raise oracle.GramBreakdown("numerically singular")
    return L.T


def test_remark_regime_pin_catches_a_breakdown_rule_at_sqrt_u():
    X, C, M = conditioned_inputs(53, 6, 3, 4, 2, 1e10)     # kappa(A) = 1e5, well below u^{-1/2}
    oracle.gram(X, 1e-14)                                  # the oracle factors it
    try:
        _gram_sqrt_u_rule(X)
    except oracle.GramBreakdown:
        return
    raise AssertionError("the sqrt(u) rule did not fire below the remark's regime")
