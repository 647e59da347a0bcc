"""GPU orthogonalization schemes (Algorithms 1-5) against the oracle.

Compared: R entry by entry, each q_i by the norm of the TT difference, and
the loss-of-orthogonality curve within 2x.  LOO values below the FP64
rounding level of the scheme itself (100 k u kappa(A_k)^p, p = 2 for
CGS/Gram, 1 for MGS, 0 for CGS2/MGS2: the matrix-case bounds of Section 3.4)
are rounding noise on both sides and are floored there before the ratio is
taken.  Tolerances on R and Q grow with kappa(A_k)^p as the schemes' own
error propagation does.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from inputs import conditioned_inputs
from gpu_util import need_gpu, dev_sum, host_cores, diff_norm

pytestmark = pytest.mark.gpu

POW = {"cgs": 2, "mgs": 1, "cgs2": 1, "mgs2": 1, "gram": 2}


def run_both(scheme, X, delta, dtype=torch.float64):
    tt = need_gpu()
    ref = oracle.orthogonalize(scheme, X, delta)
    ref_loo = oracle.loo_curve(ref.Q)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    A = [dev_sum([(a, [c.astype(npdt) for c in x]) for a, x in s], dtype) for s in X]
    Q, R, loo, st = tt.orthogonalize(scheme, A, delta)
    return ref, ref_loo, Q, R, loo, st


def compare(scheme, X, M, delta, ref, ref_loo, Q, R, loo, st, base_tol, loo_floor_u=1.1e-16):
    m = len(X)
    assert st["rounds"] == ref.rounds
    assert st["m_reached"] == m
    for k in range(1, m + 1):
        kap = math.sqrt(np.linalg.cond(M[:k, :k]))
        tol = base_tol * max(1.0, kap ** POW[scheme])
        if tol > 1e-3:
            break
        i = k - 1
        assert np.allclose(R[: i + 1, i], ref.R[: i + 1, i], rtol=0, atol=tol * max(1.0, np.abs(ref.R[:, i]).max())), (scheme, i)
        qd = diff_norm(host_cores(Q[i]), ref.Q[i]) / max(oracle.tt_norm(ref.Q[i]), 1e-300)
        assert qd <= tol, (scheme, i, qd)
    pl = {"cgs": 2, "gram": 2, "mgs": 1, "cgs2": 0, "mgs2": 0}[scheme]
    for k in range(1, m + 1):
        kap = math.sqrt(np.linalg.cond(M[:k, :k]))
        fl = 100 * k * loo_floor_u * max(1.0, kap ** pl)
        a, b = max(loo[k - 1], fl), max(ref_loo[k - 1], fl)
        assert a <= 2 * b and b <= 2 * a, (scheme, k, loo[k - 1], ref_loo[k - 1])


@pytest.mark.parametrize("scheme", ["cgs", "mgs", "cgs2", "mgs2", "gram"])
def test_schemes_small(scheme):
    X, C, M = conditioned_inputs(500, 6, 3, 5, 2, 1e4)
    ref, ref_loo, Q, R, loo, st = run_both(scheme, X, 1e-8)
    compare(scheme, X, M, 1e-8, ref, ref_loo, Q, R, loo, st, 1e-10)
    # compression gain of each q_i (Section 2): storage of the sum rounded last into q_i over q_i's
    per = 2 if scheme in ("cgs2", "mgs2") else 1
    ns = [5, 5, 5]
    size = lambda r: sum(r[k] * ns[k] * r[k + 1] for k in range(3))
    for i, q in enumerate(ref.Q):
        want = size(ref.pre_ranks[per * i + per - 1]) / size(oracle.tt_ranks(q))
        assert st["gain"][i] == pytest.approx(want, rel=1e-12), (scheme, i)


def test_mgs_twenty_vectors_order4_gram_condition_1e6():
    # m = 20 TT-vectors of order 4, n = 8, generating ranks 3, cond(Gram) = 1e6, delta = 1e-6
    X, C, M = conditioned_inputs(10000, 20, 4, 8, 3, 1e6)
    ref, ref_loo, Q, R, loo, st = run_both("mgs", X, 1e-6)
    compare("mgs", X, M, 1e-6, ref, ref_loo, Q, R, loo, st, 1e-9)


@pytest.mark.parametrize("scheme", ["cgs", "mgs", "cgs2", "mgs2", "gram"])
def test_fp32_bulk_schemes_twenty_vectors_order4(scheme):
    """The five schemes in FP32-bulk on the 20-vector order-4 workload (cond(Gram) = 1e6,
    delta = 1e-6) stored in FP32, against the oracle on the same values upcast:
    R and q within max(delta, 1e-5) kappa^p, LOO within 2x above the FP32 level."""
    X, C, M = conditioned_inputs(10000, 20, 4, 8, 3, 1e6, dtype=np.float32)
    X64 = [[(a, [c.astype(np.float64) for c in x]) for a, x in s] for s in X]
    ref = oracle.orthogonalize(scheme, X64, 1e-6)
    ref_loo = oracle.loo_curve(ref.Q)
    tt = need_gpu()
    A = [dev_sum(s, torch.float32) for s in X]
    Q, R, loo, st = tt.orthogonalize(scheme, A, 1e-6)
    compare(scheme, X, M, 1e-6, ref, ref_loo, Q, R, loo, st, 1e-5, loo_floor_u=6e-8)


def test_gram_reports_not_spd():
    tt = need_gpu()
    X, C, M = conditioned_inputs(510, 3, 3, 4, 2, 1e2)
    X.append(list(X[1]))
    A = [dev_sum(s) for s in X]
    with pytest.raises(tt.TTError) as ei:
        tt.orthogonalize("gram", A, 1e-8)
    assert ei.value.status == "TT_ENOTSPD"


def test_breakdown_on_zero_vector():
    # an exactly zero input leaves p = 0 after projection and rounding: ||p|| = 0
    tt = need_gpu()
    X, C, M = conditioned_inputs(520, 3, 3, 4, 2, 1e2)
    X.append([(0.0, x) for _, x in X[0]])
    A = [dev_sum(s) for s in X]
    for scheme in ("cgs", "mgs2"):
        with pytest.raises(tt.TTError) as ei:
            tt.orthogonalize(scheme, A, 1e-8)
        assert ei.value.status == "TT_EBREAKDOWN"


def test_rank_guard_stops_with_status():
    tt = need_gpu()
    X, C, M = conditioned_inputs(530, 5, 3, 5, 2, 1e3)
    A = [dev_sum(s) for s in X]
    with pytest.raises(tt.TTError) as ei:
        tt.orthogonalize("gram", A, 1e-8, rank_guard=5)
    assert ei.value.status == "TT_EGUARD"


def test_loo_entry_point_matches_oracle():
    tt = need_gpu()
    X, C, M = conditioned_inputs(540, 5, 3, 5, 2, 1e6)
    ref = oracle.cgs(X, 1e-4)
    from gpu_util import dev_tt
    Q = [dev_tt(q) for q in ref.Q]
    loo, G = tt.loo(Q)
    assert np.allclose(G, oracle.gram_of(ref.Q), atol=1e-13)
    assert np.allclose(loo, oracle.loo_curve(ref.Q), rtol=1e-8, atol=1e-14)


def _order6_n64_inputs():
    # m = 50 TT-vectors of order 6, n = 64, generating ranks 8, cond(Gram) = 1e10
    return conditioned_inputs(20000, 50, 6, 64, 8, 1e10)


def test_gram_fp32_dots_report_singular_gram_at_condition_1e10():
    """With FP32 dots the Gram matrix at cond 1e10 is numerically singular: reported, never hidden."""
    tt = need_gpu()
    X, C, M = _order6_n64_inputs()
    A = [dev_sum([(a, [c.astype(np.float32) for c in x]) for a, x in s], torch.float32) for s in X]
    with pytest.raises(tt.TTError) as ei:
        tt.orthogonalize("gram", A, 1e-5, rank_guard=384)
    assert ei.value.status == "TT_ENOTSPD"


@pytest.mark.parametrize("scheme,delta", [("gram", 1e-3), ("gram", 1e-7), ("cgs2", 1e-5)])
def test_order6_n64_fp64_prefix_under_rank_guard(scheme, delta):
    """FP64 CGS2 / Gram on 50 vectors: the run stops at the rank guard with TT_EGUARD and
    the completed prefix equals the oracle run on that prefix (step i only uses vectors <= i)."""
    tt = need_gpu()
    X, C, M = _order6_n64_inputs()
    A = [dev_sum(s) for s in X]
    guard = 384
    Q, R, _, st = tt.orthogonalize(scheme, A, delta, rank_guard=guard, with_loo=False, partial_on_guard=True)
    assert st.get("guard") and 1 <= st["m_reached"] < 50
    assert st["max_pre_rank"] > guard
    k = st["m_reached"]
    ref = oracle.orthogonalize(scheme, X[:k], delta)
    for i in range(k):
        kap = math.sqrt(np.linalg.cond(M[: i + 1, : i + 1]))
        tol = 1e-11 * max(1.0, kap ** POW[scheme])
        assert np.allclose(R[: i + 1, i], ref.R[: i + 1, i], rtol=0, atol=tol * max(1.0, np.abs(ref.R[:, i]).max()))
        qd = diff_norm(host_cores(Q[i]), ref.Q[i]) / oracle.tt_norm(ref.Q[i])
        assert qd <= max(tol, 2 * delta), (scheme, i, qd)


@pytest.mark.parametrize("delta", [1e-3, 1e-5, 1e-7])
def test_order6_n64_cgs2_fp32_bulk_prefix_under_rank_guard(delta):
    """FP32-bulk CGS2 on the 50 order-6 vectors (cond(Gram) = 1e10) stored in FP32, under
    the rank guard: every completed step against the oracle on the same values upcast,
    within max(delta, 1e-5) kappa(A_k)."""
    tt = need_gpu()
    X, C, M = conditioned_inputs(20000, 50, 6, 64, 8, 1e10, dtype=np.float32)
    A = [dev_sum(s, torch.float32) for s in X]
    Q, R, _, st = tt.orthogonalize("cgs2", A, delta, rank_guard=384, with_loo=False, partial_on_guard=True)
    assert st.get("guard") and 1 <= st["m_reached"] < 50
    k = st["m_reached"]
    X64 = [[(a, [c.astype(np.float64) for c in x]) for a, x in s] for s in X[:k]]
    ref = oracle.orthogonalize("cgs2", X64, delta)
    base = max(delta, 1e-5)
    for i in range(k):
        kap = math.sqrt(np.linalg.cond(M[: i + 1, : i + 1]))
        tol = base * max(1.0, kap)
        if tol > 1e-2:
            break
        assert np.allclose(R[: i + 1, i], ref.R[: i + 1, i], rtol=0, atol=tol * max(1.0, np.abs(ref.R[:, i]).max())), (i,)
        qd = diff_norm(host_cores(Q[i]), ref.Q[i]) / oracle.tt_norm(ref.Q[i])
        assert qd <= tol, (i, qd, tol)
