"""FP64 CPU oracle for randomized rounding of TT sums (TEST INFRASTRUCTURE ONLY).

The paper rounds sums of TT-vectors with the deterministic TT-round and cites
randomized rounding as the cheaper alternative when the output ranks are far
below the ranks of the sum.  This is the Randomize-then-Orthogonalize
rounding (Al Daas, Ballard, Cazeaux, Hallman, Miedlar, Pasha, Reid, Saibaba,
"Randomized algorithms for rounding in the Tensor-Train format"): with a
random Gaussian TT-vector S of ranks l_k (the sketch, drawn by the caller and
passed in), the partial contractions of x with S from the right give
W_k (R_k x l_k); then from the left Z_k = L(G_k) W_k, Q_k = orth(Z_k) becomes
core k, and M_k = Q_k^T L(G_k) is absorbed into core k+1.  With delta > 0 the
result, whose ranks are at most l_k, is rounded deterministically at delta.

Readings: the sketch is an input (its random numbers are not drawn here);
output ranks are min(l_k, p_{k-1} n_k), the columns of the thin Q of Z_k;
order d = 1 has no bond and returns the sum itself.
"""
from __future__ import annotations

import numpy as np

from .tt import tt_sum, tt_round

__all__ = ["sketch_contractions", "tt_round_rto"]


def sketch_contractions(x, sketch):
    """W_k (R_k x l_k), k = 1..d-1: cores k+1..d of x contracted with those of the sketch."""
    d = len(x)
    W = [None] * (d + 1)
    W[d] = np.ones((1, 1))
    for k in range(d - 1, 0, -1):
        # W_k[a, l] = sum_{i, b, j} X_{k+1}[a, i, b] W_{k+1}[b, j] S_{k+1}[l, i, j], as two products
        a, n, b = x[k].shape
        T = x[k].reshape(a * n, b) @ W[k + 1]                     # (a n) x l_{k+1}
        W[k] = T.reshape(a, -1) @ sketch[k].reshape(sketch[k].shape[0], -1).T
    return W


def tt_round_rto(terms, sketch, delta=0.0):
    """Randomize-then-Orthogonalize rounding of the lazy sum `terms` with the sketch TT-vector."""
    x = tt_sum(terms)
    d = len(x)
    if d == 1:
        return tt_round(x, delta) if delta > 0 else x
    W = sketch_contractions(x, sketch)
    out = []
    G = x[0]
    for k in range(d - 1):
        p0, n, R = G.shape
        L = G.reshape(p0 * n, R)
        Z = L @ W[k + 1]
        Q, _ = np.linalg.qr(Z)
        out.append(Q.reshape(p0, n, Q.shape[1]))
        M = Q.T @ L
        r1, n1, r2 = x[k + 1].shape
        G = (M @ x[k + 1].reshape(r1, n1 * r2)).reshape(M.shape[0], n1, r2)
    out.append(G)
    return tt_round(out, delta) if delta > 0 else out
