"""The Section 4 order-6 experiment on the GPU (Krylov TT-vectors of the Dirichlet
Laplacian: d = 6, n = 15, delta = 1e-5, FP64) against the oracle's run stored in
golden/order6_oracle.json (written by golden/make_order6_oracle.py, which calls only
the oracle).  The pre-round ranks reach several thousand, so the right-to-left QRs run
in column blocks and the left-to-right SVDs by block Jacobi; each scheme runs up to a
pre-round rank guard (the completed prefix is compared).

Compared on the prefix, with kappa(A_k) from the FP64 Gram matrix of the oracle's
(rank-one) inputs, the same gates as the order-3 experiment: the ranks of every q_i
while kappa(A_k) <= 1e6 (the residual of each pass is then far above the rounding noise
of the terms it is summed from); the loss of orthogonality within 2x, both floored at
100 k u kappa^p, where delta kappa^p <= 0.1 (p = 2 for CGS, 1 otherwise: the range where
the bounds of Section 3.4 fix it); beyond, finite and at most 10 k.  Past kappa ~ 1e8 the
singular values near the truncation threshold are the rounding noise of cancelling
terms, and the ranks kept there depend on the order of the arithmetic.
"""
import json
import os

import numpy as np
import pytest

import oracle
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "order6_oracle.json")
CASES = {"cgs": (35, 0), "mgs": (35, 2048), "cgs2": (35, 2048), "mgs2": (35, 2048), "householder": (20, 8192)}
POW = {"cgs": 2, "mgs": 1, "cgs2": 1, "mgs2": 1, "householder": 1}


def kappas(m):
    A = oracle.krylov_inputs([15] * 6, m)
    G = oracle.gram_of(A)
    return [float(np.sqrt(np.linalg.cond(G[:k, :k]))) for k in range(1, m + 1)]


@pytest.mark.parametrize("scheme", list(CASES))
def test_order6_experiment_prefix_matches_oracle(scheme):
    tt = need_gpu()
    with open(GOLDEN) as f:
        ref = json.load(f)["schemes"][scheme]
    m, guard = CASES[scheme]
    kap = kappas(m)
    A = tt.krylov_laplacian([15] * 6, m)
    Q, R, _, st = tt.orthogonalize(scheme, A, 1e-5, rank_guard=guard, with_loo=False, partial_on_guard=True)
    k_done = st["m_reached"]
    assert k_done >= (m if guard == 0 else 20), (scheme, k_done)
    loo = tt.loo(Q)[0]
    ref_loo = ref["loo"]
    p = POW[scheme]
    for k in range(1, k_done + 1):
        i = k - 1
        if kap[i] <= 1e6:
            assert list(Q[i].r) == ref["q_ranks"][i], (scheme, k, Q[i].r, ref["q_ranks"][i])
        if 1e-5 * kap[i] ** p <= 0.1:
            fl = 100 * k * 1.1e-16 * kap[i] ** p
            a, b = max(loo[i], fl), max(ref_loo[i], fl)
            assert a <= 2 * b and b <= 2 * a, (scheme, k, loo[i], ref_loo[i])
        else:
            assert np.isfinite(loo[i]) and loo[i] <= 10 * k, (scheme, k, loo[i])


def test_order6_gram_breaks_down_like_the_oracle():
    tt = need_gpu()
    with open(GOLDEN) as f:
        ref = json.load(f)["schemes"]["gram"]
    assert ref["status"] == "GramBreakdown"
    with pytest.raises(tt.TTError) as ei:
        tt.orthogonalize("gram", tt.krylov_laplacian([15] * 6, 35), 1e-5)
    assert ei.value.status == "TT_ENOTSPD"
