"""The stopping rule of the one-workgroup Jacobi SVD, on the CPU.

The kernel runs cyclic one-sided Jacobi (pairs of a round from the circle schedule, a pair
rotated when |<a_p, a_q>| exceeds tol sqrt(||a_p||^2 ||a_q||^2), tol = len u) and stops after a
sweep whose rotations all had |cos| of the angle between the pair below sqrt(tol): cyclic Jacobi
converges quadratically, so every pair is then orthogonal to about tol and the confirming sweep
is skipped.  Here the same iteration, in NumPy, with that rule and with the full rule (stop only
after a sweep without any rotation): the singular values agree to working precision, the final
columns are orthogonal to a few tol, and the rule saves a sweep.
"""
import numpy as np
import pytest


def circle_pair(rnd, pair, kp):
    m = kp - 1
    p, q = (m, rnd) if pair == 0 else ((rnd + pair) % m, (rnd - pair) % m)
    return (p, q) if p < q else (q, p)


def one_sided_jacobi(R, early_stop):
    A = R.copy()                              # columns of the square R factor
    n, k = A.shape
    kp = k + (k & 1)
    tol = n * 1.1102230246251565e-16
    for sweep in range(1, 65):
        rotated, big = False, False
        for rnd in range(kp - 1):
            for pair in range(kp // 2):
                p, q = circle_pair(rnd, pair, kp)
                if q >= k:
                    continue
                al, be, ga = A[:, p] @ A[:, p], A[:, q] @ A[:, q], A[:, p] @ A[:, q]
                if ga == 0 or ga * ga <= tol * tol * al * be:
                    continue
                rotated = True
                big |= ga * ga > tol * al * be
                d, g = be - al, 2.0 * ga
                t = (g if d >= 0 else -g) / (np.hypot(d, g) + abs(d))
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = c * t
                u, w = A[:, p].copy(), A[:, q].copy()
                A[:, p], A[:, q] = c * u - s * w, s * u + c * w
        if not rotated or (early_stop and not big):
            return sweep, A
    return 64, A


@pytest.mark.parametrize("k,kind", [(48, "gaussian"), (96, "graded"), (128, "gaussian")])
def test_early_stop_gives_the_converged_result(k, kind):
    g = np.random.default_rng(k)
    X = g.standard_normal((2 * k, k))
    if kind == "graded":
        X = X * 10.0 ** (-8 * np.arange(k) / (k - 1))
    R = np.linalg.qr(X, mode="r")
    s_early, A_early = one_sided_jacobi(R, True)
    s_full, A_full = one_sided_jacobi(R, False)
    ref = np.linalg.svd(R, compute_uv=False)
    for A in (A_early, A_full):
        sv = np.sort(np.linalg.norm(A, axis=0))[::-1]
        assert np.max(np.abs(sv - ref) / ref) <= 1e-13
        Q = A / np.linalg.norm(A, axis=0)
        assert np.max(np.abs(Q.T @ Q - np.eye(k))) <= 10 * k * 1.1e-16
    assert s_early < s_full
