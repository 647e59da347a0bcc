"""Test-side input construction that needs oracle arithmetic.

The orthogonalization inputs x_k = sum_{j<=k} C[k, j] t_j must have a Gram
matrix with a prescribed spectrum.  That needs the inner products of the
generating TTs t_j, which only the oracle may compute here; the resulting
coefficients are then handed unchanged to both the oracle and the HIP path.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2211_08770_amd import synth


def conditioned_inputs(seed, m, d, n, r, kappa_gram, dtype=np.float64):
    """Lazy sums x_k = sum_{j<=k} C[k, j] t_j whose Gram matrix has condition kappa_gram.

    C = B L^{-1} D with D = diag(<t_j, t_j>)^{-1/2} (unit-norm generators),
    L = chol(D G_t D) and B = chol(M), M a random correlation matrix whose
    eigenvalues are geometric on [1, 1/kappa_gram].  Then Gram(x) = M exactly
    (up to rounding), so every ||x_k|| = 1 and cond(Gram(x)) = kappa_gram.
    Each x_k carries private copies of its t_j (no sharing across vectors).
    """
    t = synth.conditioned_terms(seed, m, d, n, r, dtype=dtype)
    t64 = [[c.astype(np.float64) for c in tj] for tj in t]
    C, M = synth.mixing_coefficients(oracle.gram_of(t64), seed, kappa_gram)
    X = []
    for k in range(m):
        X.append([(float(C[k, j]), [c.copy() for c in t[j]]) for j in range(k + 1)])
    return X, C, M


def as_dense_columns(vectors):
    """Stack vectorised TT-vectors (plain or lazy sums) as matrix columns."""
    cols = []
    for v in vectors:
        if isinstance(v, list) and v and isinstance(v[0], tuple):
            v = oracle.tt_sum(v)
        cols.append(oracle.tt_full(v).ravel())
    return np.stack(cols, axis=1)
