"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers and arranges them into TT cores; it holds no
step of the TT method itself (no rounding, inner product, QR or SVD of TT data).
Seeds follow ``10000 * workload + item`` with NumPy's PCG64 generator.

Workloads (shapes mirror the ones the paper studies: order d, mode size n,
TT-ranks, number of vectors m, rounding accuracy delta):
  * ``conditioned_terms``  - generating TTs t_j for the orthogonalization inputs
    x_k = sum_{j<=k} c_kj t_j (the coefficients are fixed by the test harness,
    which needs inner products of the t_j to prescribe the Gram spectrum);
  * ``sum_of_graded_terms`` - a sum of 20 rank-10 TTs (d=8, n=32) whose j-th
    term has every core scaled by 2**-j, for single-rounding measurements;
  * ``uneven_jobs``        - independent rounding jobs with d in [4, 10],
    n in {16, 32, 64} and one internal rank R in [8, 128];
  * ``correlation_with_spectrum`` - a unit-diagonal SPD matrix with a
    prescribed eigenvalue set (Davies-Higham, via SciPy);
  * ``mixing_coefficients`` - the lower-triangular c_kj that give the x_k a
    prescribed Gram matrix, from the Gram matrix of the t_j (computed by the
    caller) and a correlation matrix: small dense linear algebra only;
  * ``serving_solver``, ``serving_vector``, ``serving_request`` - simulated
    TT-GMRES solvers (d in [5, 8], n in {32, 64, 128}, rank in [4, 32], initial
    basis of 10-39 vectors) and the new vectors their requests orthogonalize.
"""
from __future__ import annotations

import numpy as np

__all__ = ["rng", "random_tt", "sum_of_graded_terms", "conditioned_terms",
           "uneven_jobs", "correlation_with_spectrum", "geometric_spectrum", "mixing_coefficients",
           "serving_solver", "serving_vector", "serving_request"]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def random_tt(g: np.random.Generator, ns, ranks, dtype=np.float64, scale=1.0):
    """TT with i.i.d. N(0, 1) cores (times ``scale``); ranks = (1, r_1, ..., 1)."""
    d = len(ns)
    if len(ranks) != d + 1 or ranks[0] != 1 or ranks[-1] != 1:
        raise ValueError("ranks must be (1, r_1, ..., r_{d-1}, 1)")
    cores = []
    for k in range(d):
        c = g.standard_normal((ranks[k], ns[k], ranks[k + 1])) * scale
        cores.append(c.astype(dtype))
    return cores


def sum_of_graded_terms(seed=10001, nterms=20, d=8, n=32, r=10, dtype=np.float64):
    """Lazy sum of ``nterms`` random rank-r TTs; term j has every core times 2**-j.

    Returned as a list of (coef, cores) with coef = 1.  For float32 the values
    are drawn in float64 and rounded once, so both precisions can be compared
    on identical inputs (``astype(float64)`` of the float32 cores is exact).
    """
    g = rng(seed)
    ranks = [1] + [r] * (d - 1) + [1]
    terms = []
    for j in range(nterms):
        cores = random_tt(g, [n] * d, ranks, np.float64, scale=2.0 ** (-j))
        terms.append((1.0, [c.astype(dtype) for c in cores]))
    return terms


def conditioned_terms(seed, m, d, n, r, dtype=np.float64):
    """Generating TTs t_1..t_m with i.i.d. N(0, 1) cores, all ranks r."""
    g = rng(seed)
    ranks = [1] + [r] * (d - 1) + [1]
    return [[c.astype(dtype) for c in random_tt(g, [n] * d, ranks)] for _ in range(m)]


def geometric_spectrum(m, kappa):
    """m eigenvalues spread geometrically over [1, 1/kappa], scaled to sum to m."""
    if m == 1:
        return np.ones(1)
    lam = kappa ** (-np.arange(m) / (m - 1))
    return lam * (m / lam.sum())


def correlation_with_spectrum(seed, eigs):
    """Random unit-diagonal SPD matrix with eigenvalues ``eigs`` (sum = len)."""
    from scipy.stats import random_correlation
    g = rng(seed)
    M = random_correlation.rvs(np.asarray(eigs, dtype=np.float64), random_state=g, tol=1e-12)
    return 0.5 * (M + M.T)


def uneven_jobs(seed=30000, njobs=256, d_range=(4, 10), n_choices=(16, 32, 64),
                r_range=(8, 128), dtype=np.float32):
    """Independent rounding jobs: (cores, (d, n, R)) with N(0, 1) cores.

    Each job draws d ~ U{d_lo..d_hi}, one mode size n ~ U(n_choices) for all
    modes and one internal rank R ~ U{r_lo..r_hi} for every bond (bonds are
    not capped to min(prod n_<=k, prod n_>k), so rounding must cut them).
    """
    g = rng(seed)
    jobs = []
    for _ in range(njobs):
        d = int(g.integers(d_range[0], d_range[1] + 1))
        n = int(g.choice(np.asarray(n_choices)))
        R = int(g.integers(r_range[0], r_range[1] + 1))
        ranks = [1] + [R] * (d - 1) + [1]
        cores = random_tt(g, [n] * d, ranks, np.float64)
        jobs.append(([c.astype(dtype) for c in cores], (d, n, R)))
    return jobs


def serving_solver(g: np.random.Generator, d_range=(5, 8), n_choices=(32, 64, 128), r_range=(4, 32),
                   b0_range=(10, 39), bmax=40, dtype=np.float32):
    """One simulated TT-GMRES solver of the serving workload.

    Its vectors share one right part (cores 1..d-1, rank r, right-orthonormal)
    and differ in the first core U (1 x n x r), so every vector of the solver
    and every combination of them has TT-rank r: <U_a (x) P, U_b (x) P> is the
    Frobenius product <U_a, U_b>.  `firsts` holds bmax first cores that are
    orthonormal in that product; the initial basis uses the first b0.
    """
    d = int(g.integers(d_range[0], d_range[1] + 1))
    n = int(g.choice(np.asarray(n_choices)))
    r = int(g.integers(r_range[0], r_range[1] + 1))
    b0 = int(g.integers(b0_range[0], b0_range[1] + 1))
    right = []
    for k in range(1, d):
        r1 = 1 if k == d - 1 else r
        m = g.standard_normal((r, n * r1))
        q, _ = np.linalg.qr(m.T)                       # orthonormal columns: rows of the unfolding orthonormal
        right.append(q.T.reshape(r, n, r1))
    z = g.standard_normal((n * r, bmax))
    u, _ = np.linalg.qr(z)
    firsts = [u[:, j].reshape(1, n, r) for j in range(bmax)]
    return {"d": d, "n": n, "r": r, "b0": b0, "bmax": bmax, "right": right, "firsts": firsts, "dtype": dtype}


def serving_vector(g: np.random.Generator, solver, first):
    """Cores of the solver's TT whose first core is `first`."""
    return [first.astype(solver["dtype"])] + [c.astype(solver["dtype"]) for c in solver["right"]]


def serving_request(g: np.random.Generator, solver, b):
    """First core of w = sum_{j<b} c_j q_j + t (c_j ~ N(0, 1/b), t a unit random vector of the solver)."""
    n, r = solver["n"], solver["r"]
    t = g.standard_normal((1, n, r))
    t /= np.linalg.norm(t)
    c = g.standard_normal(b) / np.sqrt(max(b, 1))
    w = t.copy()
    for j in range(min(b, len(solver["firsts"]))):
        w += c[j] * solver["firsts"][j]
    return w


def mixing_coefficients(Gt, seed, kappa_gram):
    """Coefficients C (lower triangular) with x_k = sum_{j<=k} C[k, j] t_j and Gram(x) = M.

    Gt is the Gram matrix of the generators t_j.  With D = diag(Gt)^{-1/2},
    L = chol(D Gt D), M a random correlation matrix whose eigenvalues are
    geometric on [1, 1/kappa_gram] and B = chol(M): C = B L^{-1} D, so that
    C Gt C^T = M, every ||x_k|| = 1 and cond(Gram(x)) = kappa_gram.
    Returns (C, M).
    """
    m = Gt.shape[0]
    Dm = np.diag(1.0 / np.sqrt(np.diag(Gt)))
    L = np.linalg.cholesky(Dm @ Gt @ Dm)
    M = correlation_with_spectrum(seed + 7, geometric_spectrum(m, kappa_gram))
    B = np.linalg.cholesky(M)
    C = np.tril(B @ np.linalg.inv(L) @ Dm)
    return C, M
