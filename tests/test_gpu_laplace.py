"""GPU Laplacian TT-matrix, Krylov inputs and the six schemes on them (Section 4) against the oracle.

The inputs of the scheme tests come from the oracle's Krylov generator and are
handed unchanged to both sides.  Compared as in the other scheme tests: R
entry by entry and each q_i by its difference norm while tol kappa(A_k)^p stays
below 1e-3 (p = 2 CGS/Gram, 1 otherwise: a QR factor is conditioned like A_k),
and the loss-of-orthogonality curve within 2x after flooring both at the
rounding level 100 k u kappa(A_k)^p, p = 2 for CGS/Gram and 1 otherwise (the
TT roundings of a stable scheme still leave noise that grows with kappa), for
the k where delta kappa(A_k)^p <= 0.1: the range where the matrix-case bounds
of Section 3.4, with delta for u, fix the loss of orthogonality.  Beyond it the
curves jump (Section 4 attributes this to kappa, or its square, times delta no
longer being small) and only finiteness and a bound are checked.  kappa(A_k) comes from the dense vectorised inputs (n^3 = 3375
entries at order three).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import tt_full
from gpu_util import need_gpu, dev_tt, host_cores, diff_norm
from paper_2211_08770_amd import synth

pytestmark = pytest.mark.gpu

# growth of the forward error of R and Q with kappa(A_k) (a QR factor is itself conditioned like A_k),
# and of the loss of orthogonality (the bounds of Section 3.4)
POW_RQ = {"cgs": 2, "mgs": 1, "cgs2": 1, "mgs2": 1, "gram": 2, "householder": 1}
POW_LOO = {"cgs": 2, "mgs": 1, "cgs2": 0, "mgs2": 0, "gram": 2, "householder": 0}


@pytest.mark.parametrize("ns,ranks", [([15], [1, 1]), ([15, 15, 15], [1, 3, 2, 1]), ([4, 1, 6, 3], [1, 2, 2, 3, 1]),
                                      ([15] * 6, [1, 2, 4, 5, 3, 2, 1]), ([2, 3], [1, 2, 1])])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_laplacian_matches_oracle(ns, ranks, dtype):
    tt = need_gpu()
    g = synth.rng(81)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    x = [c.astype(npdt) for c in synth.random_tt(g, ns, ranks)]
    ref = oracle.tt_laplacian([c.astype(np.float64) for c in x], -0.5)
    y = tt.laplacian(dev_tt(x, dtype), -0.5)
    assert y.r == oracle.tt_ranks(ref)
    tol = 1e-13 if dtype == torch.float64 else 1e-6
    assert diff_norm(host_cores(y), ref) <= tol * oracle.tt_norm(ref)


@pytest.mark.parametrize("ns,m", [([15, 15, 15], 20), ([15] * 6, 35), ([9], 8), ([5, 7], 10)])
def test_krylov_inputs_match_oracle(ns, m):
    tt = need_gpu()
    ref = oracle.krylov_inputs(ns, m)
    A = tt.krylov_laplacian(ns, m)
    for j in range(m):
        assert A[j].r == [1] * (len(ns) + 1)
        assert diff_norm(host_cores(A[j]), ref[j]) <= 1e-11, j


def test_krylov_inputs_fp32():
    tt = need_gpu()
    ref = oracle.krylov_inputs([15, 15, 15], 12)
    A = tt.krylov_laplacian([15, 15, 15], 12, dtype=torch.float32)
    for j in range(12):
        assert diff_norm(host_cores(A[j]), ref[j]) <= 1e-5, j


def krylov_case(m):
    A = oracle.krylov_inputs([15, 15, 15], m)
    cols = np.stack([tt_full(a).ravel() for a in A], axis=1)
    kappa = [np.linalg.cond(cols[:, :k]) for k in range(1, m + 1)]
    return A, kappa


@pytest.mark.parametrize("scheme", ["cgs", "mgs", "cgs2", "mgs2", "householder"])
@pytest.mark.parametrize("delta", [1e-3, 1e-5, 1e-8])
def test_schemes_on_krylov_inputs_order3(scheme, delta):
    tt = need_gpu()
    m = 20
    A, kappa = krylov_case(m)
    ref = oracle.orthogonalize(scheme, A, delta)
    ref_loo = oracle.loo_curve(ref.Q)
    Q, R, loo, st = tt.orthogonalize(scheme, [dev_tt(a) for a in A], delta)
    assert st["rounds"] == ref.rounds and st["m_reached"] == m
    for k in range(1, m + 1):
        tol = 1e-10 * max(1.0, kappa[k - 1] ** POW_RQ[scheme])
        if tol > 1e-3:
            break
        i = k - 1
        scale = max(1.0, np.abs(ref.R[:, i]).max())
        assert np.allclose(R[: i + 1, i], ref.R[: i + 1, i], rtol=0, atol=tol * scale), (scheme, i)
        qd = diff_norm(host_cores(Q[i]), ref.Q[i]) / max(oracle.tt_norm(ref.Q[i]), 1e-300)
        assert qd <= tol, (scheme, i, qd)
    p = max(POW_LOO[scheme], 1)
    for k in range(1, m + 1):
        kap = kappa[k - 1]
        if delta * kap ** p > 0.1:
            # outside the range where the scheme's bound fixes the loss of orthogonality (the
            # jumps Section 4 attributes to kappa times delta no longer being small): finite and bounded
            assert np.isfinite(loo[k - 1]) and loo[k - 1] <= 10 * k, (scheme, k, loo[k - 1])
            continue
        fl = 100 * k * 1.1e-16 * kap ** p
        a, b = max(loo[k - 1], fl), max(ref_loo[k - 1], fl)
        assert a <= 2 * b and b <= 2 * a, (scheme, k, loo[k - 1], ref_loo[k - 1])


def test_gram_on_krylov_inputs():
    # Twenty Krylov vectors make the Gram matrix singular in FP64 (cond(G) = cond(A)^2 ~ 1e27):
    # both sides report the breakdown.  Ten vectors (cond(A_10) ~ 1e6) still factor.
    tt = need_gpu()
    A, kappa = krylov_case(20)
    with pytest.raises(oracle.GramBreakdown):
        oracle.gram(A, 1e-5)
    with pytest.raises(tt.TTError) as ei:
        tt.orthogonalize("gram", [dev_tt(a) for a in A], 1e-5)
    assert ei.value.status == "TT_ENOTSPD"
    ref = oracle.gram(A[:10], 1e-5)
    Q, R, loo, st = tt.orthogonalize("gram", [dev_tt(a) for a in A[:10]], 1e-5)
    ref_loo = oracle.loo_curve(ref.Q)
    for k in range(1, 11):
        if 1e-5 * kappa[k - 1] ** 2 > 0.1:
            assert np.isfinite(loo[k - 1]) and loo[k - 1] <= 10 * k * max(1.0, ref_loo[k - 1])
            continue
        fl = 100 * k * 1.1e-16 * max(1.0, kappa[k - 1] ** 2)
        a, b = max(loo[k - 1], fl), max(ref_loo[k - 1], fl)
        assert a <= 2 * b and b <= 2 * a, (k, loo[k - 1], ref_loo[k - 1])


def test_laplacian_rejects_aliasing_and_bad_alpha():
    tt = need_gpu()
    from paper_2211_08770_amd.tt import TT
    g = synth.rng(82)
    x = dev_tt(synth.random_tt(g, [4, 5], [1, 2, 1]))
    lib = tt._load()
    ctx = tt._ctx()
    vx = x._vec()
    big = TT(torch.empty(4 * x.data.numel(), dtype=x.dtype, device=x.data.device), x.n, [1, 1, 1])
    vb = big._vec()
    import ctypes as C
    assert lib.tt_laplacian(ctx.h, C.byref(vx), 1.0, C.byref(vx)) == -1          # out aliases x
    assert lib.tt_laplacian(ctx.h, C.byref(vx), float("nan"), C.byref(vb)) == -1  # non-finite alpha
    small = TT(torch.empty(3, dtype=x.dtype, device=x.data.device), x.n, [1, 1, 1])
    vs = small._vec()
    assert lib.tt_laplacian(ctx.h, C.byref(vx), 1.0, C.byref(vs)) == -3          # capacity
    assert lib.tt_laplacian(ctx.h, C.byref(vx), 2.0, C.byref(vb)) == 0
