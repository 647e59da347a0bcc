"""FP64 CPU oracle for the TT orthogonalization schemes (TEST INFRASTRUCTURE ONLY).

Literal transcriptions, in the paper's order and notation, of Section 3
"Orthogonalization schemes": TT-CGS (Algorithm 1), TT-MGS (Algorithm 2),
TT-CGS2 (Algorithm 3), TT-MGS2 (Algorithm 4), TT-Gram (Algorithm 5) and
TT-Householder (Algorithms 6-8, Section 3.3), plus the loss of orthogonality
of Section 3.4, equation (LOO).

Inputs are lists of lazy sums ``[(coef, cores), ...]`` (a plain TT-vector is a
one-term sum).  Sums are materialised before every dot product and rounding,
so the running vector ``p`` is exactly the unrounded TT sum of the algorithms.

Readings taken where the paper is loose:
  * column i of R holds the projections of a_i (the text of Section 3.1.1),
    so R is upper triangular with R[j, i], j <= i (Algorithm 1 prints R(i,j));
  * in CGS2/MGS2 R_1 has a zero diagonal and R[i, i] = R_2[i, i] = ||p_2||;
  * Gram forms q_i from column i of R^{-1}: q_i = sum_{k<=i} R^{-1}[k, i] a_k
    (the equation of Section 3.2; the algorithm's R^{-1}(i, j) would read the
    zero lower triangle) and q_i is not renormalised after rounding;
  * the Gram matrix counts as numerically singular (Cholesky undefined, the
    remark of Section 3.2) when a pivot L_jj^2 falls to m u G_jj or below;
  * TT-Householder: the canonical basis vector e_i is the rank-one TT-vector
    of the multi-index phi(i), first index varying fastest (Section 3.3);
    the diagonal entry takes the stable sign of the matrix construction,
    R(i,i) = -s sqrt(||a||^2 - sum_{j<i} R(j,i)^2) with s = +1 when
    <a, e_i> > 0 and -1 otherwise, so that the i-th entry of the Householder
    vector is <a, e_i> + s gamma (the TTH-vec listing prints the opposite,
    cancelling sign); the normalisation divides by the norm of the rounded
    vector w; the input of the first Householder vector is a_1 as given
    (not rounded), so one call takes 4m - 1 roundings (Table 1 counts 4m).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .tt import tt_sum, tt_dot, tt_norm, tt_round, tt_scale, tt_ranks, tt_full, RoundLog

__all__ = ["OrthoResult", "cgs", "mgs", "cgs2", "mgs2", "gram", "householder", "orthogonalize",
           "loo_curve", "gram_of", "SCHEMES", "GramBreakdown", "HouseholderBreakdown", "canonical_index",
           "canonical_tt", "tth_vec", "apply_h_vec", "cond_curve", "gs_step"]

SCHEMES = ("cgs", "mgs", "cgs2", "mgs2", "gram")


class GramBreakdown(RuntimeError):
    """The Gram matrix is numerically not positive definite (Section 3.2 remark)."""


class HouseholderBreakdown(RuntimeError):
    """A vector to reflect has no component outside the span of the earlier canonical vectors."""


@dataclass
class OrthoResult:
    Q: list
    R: np.ndarray
    rounds: int = 0
    pre_ranks: list = field(default_factory=list)    # ranks of each rounded vector before rounding
    post_ranks: list = field(default_factory=list)   # ranks after rounding
    logs: list = field(default_factory=list)
    U: list = field(default_factory=list)            # Householder TT-vectors (TT-Householder only)


def _as_sum(a):
    """Accept either a lazy sum [(coef, cores)] or a plain TT (list of arrays)."""
    if isinstance(a, list) and a and isinstance(a[0], tuple):
        return a
    return [(1.0, a)]


def _round(res, terms, delta):
    p = tt_sum(terms)
    res.pre_ranks.append(tt_ranks(p))
    lg = RoundLog()
    pr = tt_round(p, delta, log=lg)
    res.rounds += 1
    res.post_ranks.append(tt_ranks(pr))
    res.logs.append(lg)
    return pr


def cgs(A, delta):
    """TT-CGS (Algorithm 1): project a_i on every q_j, subtract, round, normalise."""
    A = [_as_sum(a) for a in A]
    m = len(A)
    R = np.zeros((m, m))
    res = OrthoResult(Q=[], R=R)
    for i in range(m):
        a_i = tt_sum(A[i])
        terms = list(A[i])
        for j in range(i):
            R[j, i] = tt_dot(a_i, res.Q[j])
            terms.append((-R[j, i], res.Q[j]))
        p = _round(res, terms, delta)
        R[i, i] = tt_norm(p)
        res.Q.append(tt_scale(1.0 / R[i, i], p))
    return res


def mgs(A, delta):
    """TT-MGS (Algorithm 2): as CGS but each projection uses the running p."""
    A = [_as_sum(a) for a in A]
    m = len(A)
    R = np.zeros((m, m))
    res = OrthoResult(Q=[], R=R)
    for i in range(m):
        terms = list(A[i])
        for j in range(i):
            p = tt_sum(terms)
            R[j, i] = tt_dot(p, res.Q[j])
            terms.append((-R[j, i], res.Q[j]))
        p = _round(res, terms, delta)
        R[i, i] = tt_norm(p)
        res.Q.append(tt_scale(1.0 / R[i, i], p))
    return res


def _two_pass(A, delta, modified):
    A = [_as_sum(a) for a in A]
    m = len(A)
    R1 = np.zeros((m, m))
    R2 = np.zeros((m, m))
    res = OrthoResult(Q=[], R=None)
    for i in range(m):
        prev_terms = list(A[i])               # p_0 = a_i
        for Rk in (R1, R2):                   # k = 1, 2
            prev = tt_sum(prev_terms)
            terms = list(prev_terms)          # p_k = p_{k-1}
            for j in range(i):
                src = tt_sum(terms) if modified else prev
                Rk[j, i] = tt_dot(src, res.Q[j])
                terms.append((-Rk[j, i], res.Q[j]))
            p = _round(res, terms, delta)
            prev_terms = [(1.0, p)]
        R2[i, i] = tt_norm(p)
        res.Q.append(tt_scale(1.0 / R2[i, i], p))
    res.R = R1 + R2
    return res


def gs_step(scheme, Q, a, delta):
    """Step i = len(Q) of TT-CGS, TT-MGS, TT-CGS2 or TT-MGS2 (Algorithms 1-4)
    against the given q_0..q_{i-1}: the projections of a (one pass, or two
    passes each rounded, R = R_1 + R_2), the rounding and the normalisation.
    Returns (q_i, column i of R as an array of i + 1 entries)."""
    passes = 2 if scheme in ("cgs2", "mgs2") else 1
    modified = scheme in ("mgs", "mgs2")
    i = len(Q)
    res = OrthoResult(Q=[], R=None)
    col = np.zeros(i + 1)
    prev_terms = list(_as_sum(a))
    for _ in range(passes):
        prev = tt_sum(prev_terms)
        terms = list(prev_terms)
        for j in range(i):
            src = tt_sum(terms) if modified else prev
            r = tt_dot(src, Q[j])
            col[j] += r
            terms.append((-r, Q[j]))
        p = _round(res, terms, delta)
        prev_terms = [(1.0, p)]
    col[i] = tt_norm(p)
    return tt_scale(1.0 / col[i], p), col


def cgs2(A, delta):
    """TT-CGS2 (Algorithm 3): two CGS passes, each rounded; R = R_1 + R_2."""
    return _two_pass(A, delta, modified=False)


def mgs2(A, delta):
    """TT-MGS2 (Algorithm 4): two MGS passes, each rounded; R = R_1 + R_2."""
    return _two_pass(A, delta, modified=True)


def gram_of(vectors):
    """Matrix of pairwise TT inner products <v_i, v_j>."""
    m = len(vectors)
    G = np.zeros((m, m))
    for i in range(m):
        for j in range(i + 1):
            G[i, j] = G[j, i] = tt_dot(vectors[i], vectors[j])
    return G


def gram(A, delta):
    """TT-Gram (Algorithm 5): G = [<a_i, a_j>], G = L L^T, R = L^T, q_i from R^{-1}."""
    A = [_as_sum(a) for a in A]
    m = len(A)
    mats = [tt_sum(a) for a in A]
    G = gram_of(mats)
    # The Cholesky factorisation is undefined once G is numerically singular
    # (Section 3.2, remark): a pivot L_jj^2 <= m u G_jj is treated as a failure.
    try:
        L = np.linalg.cholesky(G)
    except np.linalg.LinAlgError as e:
        raise GramBreakdown(str(e)) from e
    u = np.finfo(np.float64).eps / 2
    piv = np.diag(L) ** 2
    bad = np.nonzero(piv <= m * u * np.diag(G))[0]
    if bad.size:
        raise GramBreakdown(f"numerically singular Gram matrix at pivot {int(bad[0]) + 1}")
    R = L.T.copy()
    Rinv = sla.solve_triangular(R, np.eye(m), lower=False)
    res = OrthoResult(Q=[], R=R)
    for i in range(m):
        terms = []
        for k in range(i + 1):
            for c, x in A[k]:
                terms.append((Rinv[k, i] * c, x))
        res.Q.append(_round(res, terms, delta))
    return res


def canonical_index(i, ns):
    """phi(i): the multi-index (i_1, ..., i_d) of the 1-based linear index i, the
    inverse of psi(i_1, ..., i_d) = i_1 + sum_a (i_a - 1) prod_{b<a} n_b (Section 3.3)."""
    rest = i - 1
    idx = []
    for n in ns:
        idx.append(rest % n + 1)
        rest //= n
    if rest:
        raise ValueError(f"canonical index {i} exceeds the tensor size")
    return tuple(idx)


def canonical_tt(i, ns):
    """e_i = e_{i_1} x ... x e_{i_d} with (i_1, ..., i_d) = phi(i): a TT-vector of rank one."""
    cores = []
    for n, ik in zip(ns, canonical_index(i, ns)):
        c = np.zeros((1, n, 1))
        c[0, ik - 1, 0] = 1.0
        cores.append(c)
    return cores


def tth_vec(a, F, delta, res):
    """Householder TT-vector u and the first i entries r of a column of R (Algorithm 6).

    The components of a along f_1..f_{i-1} are removed and the result rounded;
    then the i-th component is replaced by r(i) = -s sqrt(||a||^2 - sum r(j)^2)
    (stable sign, module docstring), rounded again and normalised.
    """
    i = len(F)
    r = np.zeros(i)
    s = 0.0
    terms = [(1.0, a)]
    for j in range(i - 1):
        r[j] = tt_dot(a, F[j])
        s = s + r[j] ** 2
        terms.append((-r[j], F[j]))
    w = _round(res, terms, delta)
    gamma2 = tt_dot(a, a) - s
    if not gamma2 > 0.0:
        raise HouseholderBreakdown(f"no component left outside span(e_1..e_{i - 1})")
    sign = 1.0 if tt_dot(a, F[i - 1]) > 0.0 else -1.0
    r[i - 1] = -sign * np.sqrt(gamma2)
    w = _round(res, [(1.0, w), (-r[i - 1], F[i - 1])], delta)
    nw = tt_norm(w)
    if not nw > 0.0:
        raise HouseholderBreakdown("zero Householder vector")
    return tt_scale(1.0 / nw, w), r


def apply_h_vec(terms, u):
    """b = a - 2 <a, u> u (Algorithm 7) on a lazy sum: one term is appended."""
    a = tt_sum(terms)
    return list(terms) + [(-2.0 * tt_dot(a, u), u)]


def householder(A, delta):
    """TT-Householder (Algorithm 8): Householder TT-vectors u_i against the
    canonical basis, R column by column, then q_i = H_1 ... H_i e_i rounded."""
    A = [_as_sum(a) for a in A]
    m = len(A)
    ns = [c.shape[1] for c in A[0][0][1]]
    E = [canonical_tt(i, ns) for i in range(1, m + 1)]
    R = np.zeros((m, m))
    res = OrthoResult(Q=[], R=R)
    At = [list(a) for a in A]               # the running a~_j as lazy sums
    w = tt_sum(At[0])
    for i in range(m):
        u, r = tth_vec(w, E[:i + 1], delta, res)
        R[:i + 1, i] = r
        res.U.append(u)
        for j in range(i, m):
            At[j] = apply_h_vec(At[j], u)
        if i < m - 1:
            w = _round(res, At[i + 1], delta)
    for i in range(m):
        terms = [(1.0, E[i])]
        for j in range(i, -1, -1):
            terms = apply_h_vec(terms, res.U[j])
        res.Q.append(_round(res, terms, delta))
    return res


def orthogonalize(scheme, A, delta):
    fn = {"cgs": cgs, "mgs": mgs, "cgs2": cgs2, "mgs2": mgs2, "gram": gram, "householder": householder}[scheme]
    return fn(A, delta)


def loo_curve(Q):
    """||I_k - Q_k^T Q_k||_2 for k = 1..m (Section 3.4, loss of orthogonality).

    Entries of Q_k^T Q_k are TT inner products; the 2-norm of the symmetric
    matrix I - Q_k^T Q_k is its largest absolute eigenvalue.
    """
    G = gram_of(Q)
    out = []
    for k in range(1, len(Q) + 1):
        E = np.eye(k) - G[:k, :k]
        out.append(float(np.max(np.abs(np.linalg.eigvalsh(E)))))
    return np.array(out)


def cond_curve(A):
    """kappa(A_k) = sigma_max / sigma_min of the matrix whose columns are the
    vectorised a_1..a_k, k = 1..m (the conditioning that the bounds of Section
    3.4 and the plots of Section 4 are stated against), from a dense SVD of
    the full tensors (small dense dimension only)."""
    cols = [tt_full(tt_sum(_as_sum(a))).ravel() for a in A]
    Am = np.stack(cols, axis=1)
    out = []
    for k in range(1, Am.shape[1] + 1):
        s = np.linalg.svd(Am[:, :k], compute_uv=False)
        out.append(float(s[0] / s[-1]) if s[-1] > 0 else np.inf)
    return np.array(out)
