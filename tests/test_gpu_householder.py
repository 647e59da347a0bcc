"""GPU TT-Householder (Algorithms 6-8) against the oracle.

Compared: R entry by entry (signs included: the stable sign is taken on both
sides from the same FP64 inner product), each q_i by the norm of the TT
difference, the ranks of the q_i, the number of roundings (4m - 1), and the
loss-of-orthogonality curve within 2x after flooring both at the rounding
level of the arithmetic (FP64: 100 k u; FP32-bulk: 10 k times the FP32 unit).
Householder does not amplify rounding errors with the condition number of the
inputs (Section 3.4), so the tolerances are fixed multiples of the unit
round-off of the bulk arithmetic.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from inputs import conditioned_inputs
from gpu_util import need_gpu, dev_sum, dev_tt, host_cores, diff_norm
from paper_2211_08770_amd import synth

pytestmark = pytest.mark.gpu


def run_both(X, delta, dtype=torch.float64, **kw):
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    Xc = [[(a, [c.astype(npdt).astype(np.float64) for c in x]) for a, x in s] for s in X]
    ref = oracle.householder(Xc, delta)
    A = [dev_sum([(a, [c.astype(npdt) for c in x]) for a, x in s], dtype) for s in X]
    Q, R, loo, st = tt.orthogonalize("householder", A, delta, **kw)
    return ref, Q, R, loo, st


def compare(ref, Q, R, loo, st, tol, floor):
    m = len(ref.Q)
    assert st["rounds"] == ref.rounds == 4 * m - 1
    assert st["m_reached"] == m
    scale = max(1.0, float(np.abs(ref.R).max()))
    assert np.allclose(np.tril(R, -1), 0.0)
    assert np.allclose(R, ref.R, rtol=0, atol=tol * scale), float(np.abs(R - ref.R).max())
    for i in range(m):
        assert Q[i].r == oracle.tt_ranks(ref.Q[i]), i
        qd = diff_norm(host_cores(Q[i]), ref.Q[i])
        assert qd <= tol, (i, qd)
    ref_loo = oracle.loo_curve(ref.Q)
    for k in range(1, m + 1):
        fl = floor * k
        a, b = max(loo[k - 1], fl), max(ref_loo[k - 1], fl)
        assert a <= 2 * b and b <= 2 * a, (k, loo[k - 1], ref_loo[k - 1])


@pytest.mark.parametrize("seed,m,d,n,r,kappa", [(600, 5, 3, 4, 2, 1e4), (601, 6, 3, 5, 2, 1e2)])
def test_householder_fp64_small(seed, m, d, n, r, kappa):
    X, _, _ = conditioned_inputs(seed, m, d, n, r, kappa)
    ref, Q, R, loo, st = run_both(X, 1e-8)
    compare(ref, Q, R, loo, st, 1e-9, 100 * 1.1e-16)


def test_householder_twenty_vectors_order4():
    # m = 20 TT-vectors of order 4, n = 8, generating ranks 3, cond(Gram) = 1e6, delta = 1e-6
    X, _, _ = conditioned_inputs(10000, 20, 4, 8, 3, 1e6)
    ref, Q, R, loo, st = run_both(X, 1e-6)
    compare(ref, Q, R, loo, st, 1e-8, 100 * 1.1e-16)
    assert max(loo) <= 20 * 20 * 1e-6


def test_householder_fp32_bulk():
    X, _, _ = conditioned_inputs(602, 6, 3, 5, 2, 1e3)
    ref, Q, R, loo, st = run_both(X, 1e-4, dtype=torch.float32)
    compare(ref, Q, R, loo, st, 1e-4, 10 * 6e-8)


def test_householder_unequal_modes_order_one_and_single_vector():
    tt = need_gpu()
    g = synth.rng(603)
    for ns, m in (([3, 4, 2], 5), ([7], 4), ([4, 3], 1)):
        X = [[(1.0, synth.random_tt(g, ns, [1] + [2] * (len(ns) - 1) + [1])),
              (-0.5, synth.random_tt(g, ns, [1] + [1] * (len(ns) - 1) + [1]))] for _ in range(m)]
        ref, Q, R, loo, st = run_both(X, 1e-10)
        compare(ref, Q, R, loo, st, 1e-9, 100 * 1.1e-16)


def test_householder_rejects_more_vectors_than_entries():
    tt = need_gpu()
    g = synth.rng(604)
    A = [dev_tt(synth.random_tt(g, [3], [1, 1])) for _ in range(4)]
    with pytest.raises(tt.TTError) as ei:
        tt.orthogonalize("householder", A, 1e-8)
    assert ei.value.status == "TT_EINVAL"


def test_householder_rank_guard():
    tt = need_gpu()
    X, _, _ = conditioned_inputs(605, 4, 3, 4, 2, 1e2)
    A = [dev_sum(s) for s in X]
    with pytest.raises(tt.TTError) as ei:
        tt.orthogonalize("householder", A, 1e-8, rank_guard=2)
    assert ei.value.status == "TT_EGUARD"


def test_householder_full_basis_and_exact_zero_components():
    # m equal to the number of tensor entries, and inputs with exactly zero entries along the
    # canonical directions, so that the sign rule takes its "not positive" branch
    tt = need_gpu()
    ns = [2, 3]
    # a_1 = e_2 (zero along e_1), a_2 = e_1 + e_3, a_3..a_6 random: rank-one TTs and lazy sums
    e = [oracle.canonical_tt(i, ns) for i in range(1, 7)]
    g = synth.rng(606)
    X = [[(1.0, e[1])], [(1.0, e[0]), (1.0, e[2])]]
    for _ in range(4):
        X.append([(1.0, synth.random_tt(g, ns, [1, 2, 1])), (0.3, e[5])])
    ref, Q, R, loo, st = run_both(X, 1e-12)
    compare(ref, Q, R, loo, st, 1e-9, 100 * 1.1e-16)
    assert ref.R[0, 0] == pytest.approx(1.0)          # <a_1, e_1> = 0 takes s = -1: R(1,1) = +||a_1||
    assert max(loo) < 1e-10
