"""FP64 CPU oracle for the paper's input workload (TEST INFRASTRUCTURE ONLY).

Section 4 builds the vectors to orthogonalize by a Krylov process on the
discrete Laplacian of order d with Dirichlet boundary conditions, held as a
TT-matrix (the rank-two Kronecker-sum form of Kazeev and Khoromskij):
x_1 is the TT-vector of ones, a_j is x_j rounded to TT-rank one and
normalised, and x_{j+1} = -Delta_d a_j.

Readings:
  * Delta_1 is the second-difference matrix on n interior points of the unit
    interval, h = 1/(n+1): (1/h^2) tridiag(1, -2, 1), the Laplacian itself (so
    -Delta_d is positive definite); Delta_d = sum_k I x .. x Delta_1 (mode k) x .. x I.
    A scaling of Delta_1 changes no a_j (each is normalised).
  * The TT-matrix has cores [Delta_1, I], [[I, 0], [Delta_1, I]] (interior) and
    [I; Delta_1], so Delta_d x has ranks 2 r_k on interior bonds; for d = 1 it
    is Delta_1 x.  A scalar factor goes on the first core.
  * "Rounded to TT-rank one" is TT-round with the accuracy replaced by the rank
    cap one (delta = 0, max_rank = 1); "normalised" divides by the TT norm.
"""
from __future__ import annotations

import numpy as np

from .tt import tt_round, tt_norm, tt_scale

__all__ = ["laplacian_1d", "apply_along_mode", "tt_laplacian", "tt_ones", "krylov_inputs"]


def laplacian_1d(n):
    """(1/h^2) tridiag(1, -2, 1) on n interior points, h = 1/(n+1) (Dirichlet)."""
    h = 1.0 / (n + 1)
    L = np.zeros((n, n))
    for i in range(n):
        L[i, i] = -2.0
        if i > 0:
            L[i, i - 1] = 1.0
        if i + 1 < n:
            L[i, i + 1] = 1.0
    return L / (h * h)


def apply_along_mode(M, core):
    """Core (r0, n, r1) with M applied to its mode index: out[a, i, b] = sum_j M[i, j] core[a, j, b]."""
    return np.einsum("ij,ajb->aib", M, core)


def tt_laplacian(cores, alpha=1.0):
    """TT-vector of alpha * Delta_d x: the TT-matrix-by-TT-vector product, block by block."""
    d = len(cores)
    X = [np.asarray(c, dtype=np.float64) for c in cores]
    L = [laplacian_1d(c.shape[1]) for c in X]
    if d == 1:
        return [alpha * apply_along_mode(L[0], X[0])]
    out = []
    for k in range(d):
        r0, n, r1 = X[k].shape
        LX = apply_along_mode(L[k], X[k])
        if k == 0:                      # [Delta_1 X, X]
            Y = np.zeros((1, n, 2 * r1))
            Y[:, :, :r1] = LX
            Y[:, :, r1:] = X[k]
            Y *= alpha
        elif k == d - 1:                # [X; Delta_1 X]
            Y = np.zeros((2 * r0, n, 1))
            Y[:r0] = X[k]
            Y[r0:] = LX
        else:                           # [[X, 0], [Delta_1 X, X]]
            Y = np.zeros((2 * r0, n, 2 * r1))
            Y[:r0, :, :r1] = X[k]
            Y[r0:, :, :r1] = LX
            Y[r0:, :, r1:] = X[k]
        out.append(Y)
    return out


def tt_ones(ns):
    """The TT-vector of ones: rank one, every core all ones."""
    return [np.ones((1, n, 1)) for n in ns]


def krylov_inputs(ns, m):
    """a_1..a_m: x_1 = ones, a_j = x_j rounded to rank one and normalised, x_{j+1} = -Delta_d a_j."""
    x = tt_ones(ns)
    A = []
    for j in range(m):
        a = tt_round(x, 0.0, max_rank=1)
        a = tt_scale(1.0 / tt_norm(a), a)
        A.append(a)
        if j + 1 < m:
            x = tt_laplacian(a, -1.0)
    return A
