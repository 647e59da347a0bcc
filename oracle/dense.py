"""Dense-matrix orthogonalization schemes used to pin the TT oracle (TEST INFRASTRUCTURE ONLY).

These are the classical matrix algorithms the paper generalises (Section 3:
CGS, MGS and their re-orthogonalised forms in 3.1, the Gram approach in 3.2).
Columns of ``A`` are the vectorised tensors.  With a rounding accuracy driven
to zero, each TT scheme must reproduce its matrix counterpart.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = ["dcgs", "dmgs", "dcgs2", "dmgs2", "dgram", "dense_orthogonalize", "dloo"]


def dcgs(A):
    n, m = A.shape
    Q = np.zeros((n, m))
    R = np.zeros((m, m))
    for i in range(m):
        p = A[:, i].copy()
        for j in range(i):
            R[j, i] = A[:, i] @ Q[:, j]
            p -= R[j, i] * Q[:, j]
        R[i, i] = np.linalg.norm(p)
        Q[:, i] = p / R[i, i]
    return Q, R


def dmgs(A):
    n, m = A.shape
    Q = np.zeros((n, m))
    R = np.zeros((m, m))
    for i in range(m):
        p = A[:, i].copy()
        for j in range(i):
            R[j, i] = p @ Q[:, j]
            p -= R[j, i] * Q[:, j]
        R[i, i] = np.linalg.norm(p)
        Q[:, i] = p / R[i, i]
    return Q, R


def _d2(A, modified):
    n, m = A.shape
    Q = np.zeros((n, m))
    R1 = np.zeros((m, m))
    R2 = np.zeros((m, m))
    for i in range(m):
        prev = A[:, i].copy()
        for Rk in (R1, R2):
            p = prev.copy()
            for j in range(i):
                src = p if modified else prev
                Rk[j, i] = src @ Q[:, j]
                p -= Rk[j, i] * Q[:, j]
            prev = p
        R2[i, i] = np.linalg.norm(prev)
        Q[:, i] = prev / R2[i, i]
    return Q, R1 + R2


def dcgs2(A):
    return _d2(A, False)


def dmgs2(A):
    return _d2(A, True)


def dgram(A):
    G = A.T @ A
    L = np.linalg.cholesky(G)
    R = L.T
    Q = sla.solve_triangular(R, A.T, lower=False, trans="T").T   # Q = A R^{-1}
    return Q, R


def dense_orthogonalize(scheme, A):
    return {"cgs": dcgs, "mgs": dmgs, "cgs2": dcgs2, "mgs2": dmgs2, "gram": dgram}[scheme](A)


def dloo(Q):
    out = []
    for k in range(1, Q.shape[1] + 1):
        out.append(float(np.linalg.norm(np.eye(k) - Q[:, :k].T @ Q[:, :k], 2)))
    return np.array(out)
