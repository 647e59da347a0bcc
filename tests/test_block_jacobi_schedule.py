"""Convergence of the block one-sided Jacobi schedule that the block SVD kernels run, on the CPU.

The kernels stop after at most 64 outer sweeps.  Here the same schedule is run in NumPy: A = R^T;
columns set aside when their joint energy is at most (2 sqrt(k) u ||A||_F)^2; the active columns
in blocks of 32; each round of the circle schedule on the blocks takes every disjoint pair of
blocks, forms the 64 x 64 Gram matrix of its columns, skips it when every pair of columns is
orthogonal to relative precision N u, and otherwise diagonalises it by at most two sweeps of
cyclic two-sided Jacobi (rounds of 32 disjoint pairs) and rotates the 64 columns by the
accumulated V; a sweep in which no pair of blocks rotated ends the iteration.  The column norms
are then the singular values.

This checks the schedule, not the kernels (their parity tests compare the rounding with the
oracle's): on random, geometric (1 to 1e-10) and clustered spectra the iteration ends in a few
sweeps with singular values to working precision.  Run at larger sizes, the same emulation needs
10-11 sweeps at 512 rows and 11-13 at 1024, so the cap of 64 leaves a wide margin.
"""
import numpy as np
import pytest

BB, PW = 32, 64


def circle_pair(rnd, pair, kp):
    m = kp - 1
    p, q = (m, rnd) if pair == 0 else ((rnd + pair) % m, (rnd - pair) % m)
    return (p, q) if p < q else (q, p)


def inner_jacobi(G, tol2, sweeps):
    V = np.eye(PW)
    schedule = [[circle_pair(r, i, PW) for i in range(PW // 2)] for r in range(PW - 1)]
    for _ in range(sweeps):
        rotated = False
        for pairs in schedule:
            P = np.array([p for p, _ in pairs])
            Q = np.array([q for _, q in pairs])
            al, be, ga = G[P, P], G[Q, Q], G[P, Q]
            do = (ga != 0) & (ga * ga > tol2 * al * be)
            if not do.any():
                continue
            rotated = True
            d, g2 = be - al, 2.0 * np.where(do, ga, 1.0)
            t = np.where(d >= 0, g2, -g2) / (np.sqrt(d * d + g2 * g2) + np.abs(d))
            c = np.where(do, 1.0 / np.sqrt(1.0 + t * t), 1.0)
            s = np.where(do, c * t, 0.0)
            for M, rows in ((G, True), (G, False), (V, False)):
                u, w = (M[P, :].copy(), M[Q, :].copy()) if rows else (M[:, P].copy(), M[:, Q].copy())
                a, b = (c[:, None], s[:, None]) if rows else (c, s)
                if rows:
                    M[P, :], M[Q, :] = a * u - b * w, b * u + a * w
                else:
                    M[:, P], M[:, Q] = a * u - b * w, b * u + a * w
        if not rotated:
            break
    return V


def block_jacobi(R, inner=2, max_sweeps=64):
    A = R.T.copy()
    N, k = A.shape
    u = 2.0 ** -53
    nrm2 = (A * A).sum(0)
    tau2 = (2 * np.sqrt(k) * u) ** 2 * nrm2.sum()
    order = np.lexsort((np.arange(k), nrm2))
    aside = set(order[np.cumsum(nrm2[order]) <= tau2].tolist())
    act = [j for j in range(k) if j not in aside and nrm2[j] != 0]
    nb = (len(act) + BB - 1) // BB
    nbp = nb + (nb & 1)
    tol2 = (N * 1.1102230246251565e-16) ** 2
    for sweep in range(max_sweeps):
        if nb < 2 and sweep > 0:
            return sweep, A
        rotated = 0
        for rnd in range(max(nbp - 1, 1)):
            for pair in range(max(nbp // 2, 1)):
                bp, bq = circle_pair(rnd, pair, nbp) if nbp >= 2 else (0, 1)
                slots = list(range(bp * BB, bp * BB + BB)) + list(range(bq * BB, bq * BB + BB))
                live = np.array([a < len(act) for a in slots])
                idx = np.array([act[a] for a in slots if a < len(act)])
                X = np.zeros((N, PW))
                X[:, live] = A[:, idx]
                G = X.T @ X
                iu = np.triu_indices(PW, 1)
                ga, al, be = G[iu], np.diag(G)[iu[0]], np.diag(G)[iu[1]]
                if not np.any((ga != 0) & (ga * ga > tol2 * al * be)):
                    continue
                rotated += 1
                A[:, idx] = (X @ inner_jacobi(G, tol2, 40 if nb < 2 else inner))[:, live]
        if rotated == 0:
            return sweep + 1, A
    return max_sweeps, A


def r_factor(g, k, kind):
    M = 2 * k
    if kind == "gaussian":
        X = g.standard_normal((M, k))
    elif kind == "geometric":
        U, _ = np.linalg.qr(g.standard_normal((M, k)))
        V, _ = np.linalg.qr(g.standard_normal((k, k)))
        X = (U * 10.0 ** (-10 * np.arange(k) / (k - 1))) @ V.T
    else:   # clustered scales, as a sum of rank-8 terms scaled by 2^-(j mod 7)
        X = sum(2.0 ** -(j % 7) * (g.standard_normal((M, 8)) @ g.standard_normal((8, k))) for j in range(k // 8))
    return np.linalg.qr(X, mode="r")


@pytest.mark.parametrize("k", [128, 256])
@pytest.mark.parametrize("kind", ["gaussian", "geometric", "clustered"])
def test_schedule_converges_well_within_the_sweep_cap(k, kind):
    R = r_factor(np.random.default_rng(k + len(kind)), k, kind)
    sweeps, A = block_jacobi(R)
    sv = np.sort(np.linalg.norm(A, axis=0))[::-1]
    ref = np.linalg.svd(R, compute_uv=False)
    assert sweeps <= 16, sweeps
    assert np.max(np.abs(sv - ref)) <= 1e-12 * ref[0]
