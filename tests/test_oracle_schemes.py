"""Pins of the oracle's orthogonalization schemes (Algorithms 1-5) and LOO.

Independent references: the dense matrix algorithms on vectorised inputs
(to which each TT scheme reduces when the rounding accuracy goes to zero),
structural invariants (round counts of Table 1, rank additivity of
Section 2, the rank bound of the Gram scheme in Section 3.2), and the dense
2-norm for the loss of orthogonality.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import dense, tt_full, tt_ranks, tt_sum
from paper_2211_08770_amd import synth
from inputs import conditioned_inputs, as_dense_columns

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_inputs(seed=40, m=5, ns=(3, 4, 3), r=2, kappa=1e3):
    X, C, M = conditioned_inputs(seed, m, len(ns), ns[0], r, kappa)
    return X


POWER = {"cgs": 2, "mgs": 1, "cgs2": 0, "mgs2": 0, "gram": 2}


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_scheme_matches_dense_matrix_version(scheme):
    X, C, M = conditioned_inputs(41, 5, 3, 4, 2, 1e4)
    A = as_dense_columns(X)
    kappa = math.sqrt(1e4)
    res = oracle.orthogonalize(scheme, X, 1e-14)
    Qd, Rd = dense.dense_orthogonalize(scheme, A)
    Qt = as_dense_columns(res.Q)
    tol = 1e-11 * max(1.0, kappa ** POWER[scheme])
    assert np.allclose(res.R, Rd, rtol=0, atol=tol)
    assert np.allclose(Qt, Qd, rtol=0, atol=tol)


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_orthonormal_input_gives_identity(scheme):
    # Orthonormal TT inputs: R = I and Q = A.
    g = synth.rng(42)
    ns = (3, 4, 3)
    Qd, _ = np.linalg.qr(g.standard_normal((36, 4)))
    A = []
    for i in range(4):
        cores, _ = oracle.tt_svd(Qd[:, i].reshape(ns), 0.0)
        A.append(cores)
    res = oracle.orthogonalize(scheme, A, 1e-13)
    assert np.allclose(res.R, np.eye(4), atol=1e-12)
    assert np.allclose(as_dense_columns(res.Q), Qd, atol=1e-12)


def test_round_counts_follow_table1():
    with open(os.path.join(GOLDEN, "table1_round_counts.json")) as f:
        table = json.load(f)
    X = small_inputs(m=4)
    for scheme in oracle.SCHEMES:
        res = oracle.orthogonalize(scheme, X, 1e-8)
        assert res.rounds == table["rounds_per_vector"][scheme] * 4, scheme


@pytest.mark.parametrize("scheme", ["cgs", "mgs"])
def test_pre_round_rank_is_sum_of_ranks(scheme):
    # p = a_i - sum_j R(j,i) q_j: its k-th rank is rank_k(a_i) + sum_j rank_k(q_j).
    X = small_inputs(seed=43, m=4)
    res = oracle.orthogonalize(scheme, X, 1e-6)
    for i in range(4):
        ra = tt_ranks(tt_sum(X[i]))
        expect = [a + sum(tt_ranks(res.Q[j])[k] for j in range(i)) for k, a in enumerate(ra)]
        expect[0] = expect[-1] = 1
        assert res.pre_ranks[i] == expect


def test_gram_rank_bound():
    # Section 3.2: before rounding q_i has rank sum_{k<=i} rank(a_k); after rounding at most that.
    X = small_inputs(seed=44, m=4)
    res = oracle.gram(X, 1e-6)
    for i in range(4):
        bound = [sum(tt_ranks(tt_sum(X[k]))[b] for k in range(i + 1)) for b in range(4)]
        bound[0] = bound[-1] = 1
        assert res.pre_ranks[i] == bound
        assert all(p <= q for p, q in zip(res.post_ranks[i], bound))


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_qr_residual_is_of_order_delta(scheme):
    delta = 1e-6
    X = small_inputs(seed=45, m=5, kappa=1e2)
    res = oracle.orthogonalize(scheme, X, delta)
    A = as_dense_columns(X)
    Q = as_dense_columns(res.Q)
    for i in range(5):
        r = A[:, i] - Q[:, : i + 1] @ res.R[: i + 1, i]
        assert np.linalg.norm(r) <= 20 * (i + 1) * delta * np.linalg.norm(A[:, i])
    assert np.allclose(np.tril(res.R, -1), 0)


def test_loo_matches_dense_two_norm():
    X = small_inputs(seed=46, m=5, kappa=1e6)
    res = oracle.cgs(X, 1e-4)
    Q = as_dense_columns(res.Q)
    assert np.allclose(oracle.loo_curve(res.Q), dense.dloo(Q), rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_loo_bounds_with_delta_in_place_of_u(scheme):
    # Table 1 (TT column) with the reading of the text for MGS: LOO = O(delta
    # kappa^2) for CGS/Gram, O(delta kappa) for MGS (Table 1 prints kappa^2 for it
    # while the text says it follows kappa), O(delta) for CGS2/MGS2.  Checked only
    # where delta * kappa^p <= 0.1.
    delta = 1e-8
    X, C, M = conditioned_inputs(47, 6, 3, 4, 2, 1e4)
    kappa_g = np.linalg.cond(M)
    res = oracle.orthogonalize(scheme, X, delta)
    loo = oracle.loo_curve(res.Q)
    for k in range(1, 7):
        kap = math.sqrt(np.linalg.cond(M[:k, :k]))
        p = {"cgs": 2, "gram": 2, "mgs": 1, "cgs2": 0, "mgs2": 0}[scheme]
        if delta * kap ** p <= 0.1:
            assert loo[k - 1] <= 10 * k * delta * max(1.0, kap ** p) + 1e-13, (scheme, k)
    assert kappa_g == pytest.approx(1e4, rel=1e-6)


def test_gram_breakdown_on_dependent_input():
    X = small_inputs(seed=48, m=3)
    X.append([(1.0, tt_sum(X[1]))])          # exact duplicate of a_2
    with pytest.raises(oracle.GramBreakdown):
        oracle.gram(X, 1e-8)


def test_mgs_projection_equals_component_form():
    # The MGS projection of the unrounded running sum equals
    # <a_i, q_j> - sum_{l<j} R(l,i) <q_l, q_j>, up to reordering of rounding.
    X = small_inputs(seed=49, m=5, kappa=1e4)
    res = oracle.mgs(X, 1e-6)
    GQ = oracle.gram_of(res.Q)
    for i in range(1, 5):
        a = tt_sum(X[i])
        for j in range(i):
            comp = oracle.tt_dot(a, res.Q[j]) - sum(res.R[l, i] * GQ[l, j] for l in range(j))
            scale = abs(oracle.tt_dot(a, res.Q[j])) + sum(abs(res.R[l, i] * GQ[l, j]) for l in range(j))
            assert abs(comp - res.R[j, i]) <= 1e-13 * max(scale, 1.0)


def test_conditioned_inputs_have_prescribed_gram():
    X, C, M = conditioned_inputs(50, 6, 4, 3, 2, 1e6)
    A = as_dense_columns(X)
    G = A.T @ A
    assert np.allclose(G, M, atol=1e-9)
    assert np.linalg.cond(G) == pytest.approx(1e6, rel=1e-3)


def test_cond_curve_pins():
    """kappa(A_k): 1 on orthonormal columns, max/min scale on orthogonal scaled
    columns, sqrt(cond(Gram)) on the conditioned inputs (their Gram matrix is
    the prescribed correlation matrix)."""
    g = synth.rng(43)
    ns = (3, 4, 3)
    Qd, _ = np.linalg.qr(g.standard_normal((36, 5)))
    A = [oracle.tt_svd(Qd[:, i].reshape(ns), 0.0)[0] for i in range(5)]
    assert np.allclose(oracle.cond_curve(A), 1.0, atol=1e-12)
    scales = [1.0, 0.5, 4.0, 1e-3, 2.0]
    B = [oracle.tt_svd(scales[i] * Qd[:, i].reshape(ns), 0.0)[0] for i in range(5)]
    want = [max(scales[:k]) / min(scales[:k]) for k in range(1, 6)]
    assert np.allclose(oracle.cond_curve(B), want, rtol=1e-10)
    X, C, M = conditioned_inputs(44, 8, 3, 4, 2, 1e6)
    kap = oracle.cond_curve(X)
    assert abs(kap[-1] / math.sqrt(1e6) - 1.0) < 1e-6
    assert np.all(np.diff(kap) >= -1e-9 * kap[1:])   # adding columns never lowers kappa


@pytest.mark.parametrize("scheme", ["cgs", "mgs", "cgs2", "mgs2"])
def test_gs_step_reproduces_the_full_scheme(scheme):
    """One Gram-Schmidt step against the scheme's own earlier q_j gives the same q_i and
    column i of R as the full run (the step of Algorithms 1-4, R(i,i) = ||p|| of the last pass)."""
    X, C, M = conditioned_inputs(51, 5, 3, 4, 2, 1e4)
    res = oracle.orthogonalize(scheme, X, 1e-6)
    for i in range(5):
        q, col = oracle.gs_step(scheme, res.Q[:i], X[i], 1e-6)
        assert np.array_equal(col, res.R[: i + 1, i])
        assert all(np.array_equal(a, b) for a, b in zip(q, res.Q[i]))


@pytest.mark.parametrize("kappa_gram", [1e10, 1e14])
def test_gram_factors_below_the_remark_regime(kappa_gram):
    """Section 3.2's remark puts the failure of the Cholesky factorisation of G at kappa(A)
    above about u^{-1/2} (kappa(G) = kappa(A)^2 near 1/u).  Below it the oracle's breakdown
    rule (a pivot at the rounding level, L_jj^2 <= m u G_jj) must not fire: at kappa(G) = 1e10
    and 1e14 (kappa(A) = 1e5 and 1e7, under u^{-1/2} = 6.7e7) TT-Gram completes and R^T R
    reproduces the dense Gram matrix of the vectorised inputs.  A rule at the square root of
    the round-off, sqrt(u) G_jj, would already stop the first case."""
    X, C, M = conditioned_inputs(53, 6, 3, 4, 2, kappa_gram)
    res = oracle.gram(X, 1e-14)
    A = as_dense_columns(X)
    G = A.T @ A
    assert np.all(np.diag(res.R) > 0) and np.allclose(np.tril(res.R, -1), 0)
    assert np.linalg.norm(res.R.T @ res.R - G) <= 1e-12 * np.linalg.norm(G)
    assert np.linalg.cond(G) == pytest.approx(kappa_gram, rel=1e-2)


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_dense_schemes_equal_lapack_qr_on_well_conditioned_columns(scheme):
    """The dense matrix schemes that pin the TT oracle are pinned themselves to LAPACK's
    Householder QR (numpy.linalg.qr with the signs chosen to make the diagonal of R positive,
    the convention every Gram-Schmidt form and the Cholesky factor share): on columns of
    condition number about 10, Q and R agree to rounding for every scheme."""
    g = synth.rng(54)
    A = g.standard_normal((40, 7)) @ np.diag([1.0, 2.0, 0.5, 3.0, 1.0, 0.8, 1.5])
    assert np.linalg.cond(A) < 30
    Q, R = dense.dense_orthogonalize(scheme, A)
    Ql, Rl = np.linalg.qr(A)
    s = np.sign(np.diag(Rl))
    Ql, Rl = Ql * s, s[:, None] * Rl
    assert np.allclose(R, Rl, rtol=0, atol=1e-12 * np.linalg.norm(A))
    assert np.allclose(Q, Ql, rtol=0, atol=1e-12)


def test_dense_loo_is_the_largest_eigenvalue_magnitude():
    """dloo(Q)[k-1] = ||I - Q_k^T Q_k||_2 (Section 3.4): on a non-orthonormal Q it equals the
    largest absolute eigenvalue of the symmetric I - Q_k^T Q_k (LAPACK's symmetric eigensolver,
    a route independent of the SVD behind the 2-norm)."""
    g = synth.rng(55)
    Q = g.standard_normal((30, 6)) / math.sqrt(30)
    got = dense.dloo(Q)
    for k in range(1, 7):
        E = np.eye(k) - Q[:, :k].T @ Q[:, :k]
        assert got[k - 1] == pytest.approx(np.abs(np.linalg.eigvalsh(E)).max(), rel=1e-12)
