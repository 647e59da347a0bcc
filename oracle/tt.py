"""FP64 CPU oracle for the TT primitives (TEST INFRASTRUCTURE ONLY).

This module is the reference that the HIP path is checked against. Only the
test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` (its CPU part: host timings of this oracle and checks of GPU
results against it) may import it; the product path never does.

Everything is plain NumPy in float64, written to be read against the paper
(Coulaud, Giraud, Iannacito, "On some orthogonalization schemes in Tensor
Train format", Inria RR-9491, Section 2 "Notation and TT-format").

A TT-vector is a Python list of cores; core k is an array of shape
``(r_{k-1}, n_k, r_k)`` with ``r_0 = r_d = 1``.  A lazy sum is a list of
``(coef, cores)`` pairs and is materialised with :func:`tt_sum`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "tt_ranks", "tt_full", "tt_dot", "tt_norm", "tt_axpy", "tt_sum", "tt_scale",
    "tt_round", "RoundLog", "select_rank", "tt_svd", "tt_copy", "tt_rank_caps",
    "compression_ratio", "compression_gain", "tt_orth_rl",
]


def _f64(cores):
    return [np.asarray(c, dtype=np.float64) for c in cores]


def tt_copy(cores):
    return [np.array(c, dtype=np.float64, copy=True) for c in cores]


def tt_ranks(cores):
    """TT-ranks (r_0, ..., r_d) of a TT-vector (Section 2, TT representation)."""
    return [cores[0].shape[0]] + [c.shape[2] for c in cores]


def tt_rank_caps(ns):
    """Largest possible rank of each bond: min(prod n_{<=k}, prod n_{>k})."""
    d = len(ns)
    caps = [1]
    for k in range(1, d):
        left = math.prod(ns[:k])
        right = math.prod(ns[k:])
        caps.append(min(left, right))
    caps.append(1)
    return caps


def tt_full(cores):
    """Dense tensor of a TT-vector.

    Each entry is the product of the slice matrices X_1(i_1) ... X_d(i_d)
    (Section 2, element-wise form of the TT representation); contracting the
    cores one bond at a time evaluates all those products together.
    """
    cores = _f64(cores)
    ns = [c.shape[1] for c in cores]
    acc = cores[0].reshape(cores[0].shape[1], cores[0].shape[2])  # (n_1, r_1)
    for c in cores[1:]:
        r0, n, r1 = c.shape
        acc = acc @ c.reshape(r0, n * r1)          # (prod n, n * r1)
        acc = acc.reshape(-1, r1)
    return acc.reshape(ns)


def tt_dot(x, y):
    """Euclidean inner product <x, y> of two TT-vectors (Section 2).

    Left-to-right contraction W_k = sum_i X_k(i)^T W_{k-1} Y_k(i), W_0 = 1,
    so <x, y> = W_d.
    """
    x = _f64(x)
    y = _f64(y)
    if len(x) != len(y):
        raise ValueError("order mismatch")
    W = np.ones((1, 1))
    for X, Y in zip(x, y):
        if X.shape[1] != Y.shape[1]:
            raise ValueError("mode size mismatch")
        Wn = np.zeros((X.shape[2], Y.shape[2]))
        for i in range(X.shape[1]):
            Wn += X[:, i, :].T @ W @ Y[:, i, :]
        W = Wn
    return float(W[0, 0])


def tt_norm(x):
    """Frobenius norm of a TT-vector, sqrt(<x, x>)."""
    v = tt_dot(x, x)
    return math.sqrt(max(v, 0.0))


def tt_scale(alpha, x):
    """alpha * x, applied to the last core (the normalisation step of Algs 1-4)."""
    out = tt_copy(x)
    out[-1] = out[-1] * alpha
    return out


def tt_sum(terms):
    """Materialise a lazy sum  sum_c coef_c * x^(c)  as one TT-vector.

    TT addition (Section 2): ranks add; the first core is the horizontal
    concatenation, the middle cores are block diagonal, the last core is the
    vertical concatenation.  Each coefficient multiplies its term's first core.
    """
    terms = [(float(a), _f64(x)) for a, x in terms]
    if not terms:
        raise ValueError("empty sum")
    d = len(terms[0][1])
    ns = [c.shape[1] for c in terms[0][1]]
    for _, x in terms:
        if len(x) != d or [c.shape[1] for c in x] != ns:
            raise ValueError("shape mismatch in sum")
    if d == 1:
        return [sum(a * x[0] for a, x in terms).reshape(1, ns[0], 1)]
    ranks = [sum(x[k].shape[2] for _, x in terms) for k in range(d - 1)]
    out = []
    # first core: [a_1 X_1 | a_2 Y_1 | ...]
    first = np.zeros((1, ns[0], ranks[0]))
    off = 0
    for a, x in terms:
        r = x[0].shape[2]
        first[:, :, off:off + r] = a * x[0]
        off += r
    out.append(first)
    for k in range(1, d - 1):
        core = np.zeros((ranks[k - 1], ns[k], ranks[k]))
        o0 = o1 = 0
        for _, x in terms:
            r0, _, r1 = x[k].shape
            core[o0:o0 + r0, :, o1:o1 + r1] = x[k]
            o0 += r0
            o1 += r1
        out.append(core)
    last = np.zeros((ranks[d - 2], ns[d - 1], 1))
    off = 0
    for _, x in terms:
        r = x[d - 1].shape[0]
        last[off:off + r] = x[d - 1]
        off += r
    out.append(last)
    return out


def tt_axpy(alpha, x, y):
    """z = alpha * x + y as a materialised TT-vector (ranks add, Section 2)."""
    return tt_sum([(alpha, x), (1.0, y)])


def select_rank(sigma, eps, max_rank=None):
    """Smallest t >= 1 with sqrt(sum_{i>t} sigma_i^2) <= eps.

    ``sigma`` is sorted in decreasing order.  The tail sums are accumulated
    from the smallest singular value upward.  Returns ``(t, margin)`` where
    ``margin = min(tail_{t-1} / eps, eps / tail_t)`` measures how far the
    decision is from a tie (inf when it is not close to any).
    """
    s = np.asarray(sigma, dtype=np.float64)
    m = s.size
    tail2 = np.zeros(m + 1)                 # tail2[t] = sum_{i >= t} s_i^2 (0-based)
    for i in range(m - 1, -1, -1):
        tail2[i] = tail2[i + 1] + s[i] * s[i]
    eps2 = eps * eps
    t = m
    for cand in range(1, m + 1):
        if tail2[cand] <= eps2:
            t = cand
            break
    if max_rank is not None and max_rank > 0:
        t = min(t, int(max_rank))
    t = max(t, 1)
    above = math.sqrt(tail2[t - 1]) if t - 1 >= 1 else math.inf  # rank t-1 was insufficient
    below = math.sqrt(tail2[t]) if t < m else 0.0
    if eps <= 0:
        margin = math.inf
    else:
        r1 = above / eps if above != math.inf else math.inf
        r2 = eps / below if below > 0 else math.inf
        margin = min(r1, r2)
    return t, margin


@dataclass
class RoundLog:
    """Diagnostics of one rounding: norm, threshold, spectra, margins, ranks."""
    norm: float = 0.0
    eps: float = 0.0
    sigmas: list = field(default_factory=list)
    margins: list = field(default_factory=list)
    rl_ranks: list = field(default_factory=list)
    out_ranks: list = field(default_factory=list)
    in_ranks: list = field(default_factory=list)


def tt_orth_rl(cores):
    """Right-to-left orthogonalisation sweep; returns (cores, R-factors).

    For k = d..2: QR of the transposed right unfolding of core k; core k
    becomes right-orthonormal and the R factor is absorbed into core k-1.
    After the sweep ||x|| = ||G_1||_F.
    """
    G = tt_copy(cores)
    d = len(G)
    Rs = [None] * d
    for k in range(d - 1, 0, -1):
        r0, n, r1 = G[k].shape
        Y = G[k].reshape(r0, n * r1).T                 # (n r1) x r0
        Q, R = np.linalg.qr(Y, mode="reduced")
        s = Q.shape[1]
        G[k] = Q.T.reshape(s, n, r1)
        a, m, _ = G[k - 1].shape
        G[k - 1] = (G[k - 1].reshape(a * m, r0) @ R.T).reshape(a, m, s)
        Rs[k] = R
    return G, Rs


def tt_round(cores, delta, max_rank=None, log=None):
    """TT-round(x, delta) (Section 2; the algorithm the paper cites).

    Two sweeps:
      1. right-to-left orthogonalisation by QR (``tt_orth_rl``);
      2. left-to-right truncated SVD of each left unfolding with the per-bond
         threshold eps = delta / sqrt(d-1) * ||x||, where ||x|| = ||G_1||_F
         after step 1.  The kept rank is the smallest with tail <= eps,
         optionally capped by ``max_rank``.
    Returns a new TT-vector whose cores 1..d-1 are left-orthonormal, so that
    ||x_tilde|| = ||G_d||_F and ||x - x_tilde|| <= delta ||x||.
    """
    cores = _f64(cores)
    d = len(cores)
    if delta < 0 or not np.isfinite(delta):
        raise ValueError("delta must be finite and >= 0")
    if log is not None:
        log.in_ranks = tt_ranks(cores)
    if d == 1:
        out = tt_copy(cores)
        if log is not None:
            log.norm = float(np.linalg.norm(out[0]))
            log.out_ranks = tt_ranks(out)
        return out
    G, _ = tt_orth_rl(cores)
    if log is not None:
        log.rl_ranks = tt_ranks(G)
    nrm = float(np.linalg.norm(G[0]))
    if log is not None:
        log.norm = nrm
    if nrm == 0.0:
        out = [np.zeros((1, c.shape[1], 1)) for c in cores]
        if log is not None:
            log.out_ranks = tt_ranks(out)
        return out
    eps = delta / math.sqrt(d - 1) * nrm
    if log is not None:
        log.eps = eps
    for k in range(d - 1):
        a, n, b = G[k].shape
        U, S, Vt = np.linalg.svd(G[k].reshape(a * n, b), full_matrices=False)
        t, margin = select_rank(S, eps, max_rank)
        if log is not None:
            log.sigmas.append(S.copy())
            log.margins.append(margin)
        G[k] = U[:, :t].reshape(a, n, t)
        _, n1, c1 = G[k + 1].shape
        G[k + 1] = ((S[:t, None] * Vt[:t]) @ G[k + 1].reshape(b, n1 * c1)).reshape(t, n1, c1)
    if log is not None:
        log.out_ranks = tt_ranks(G)
    return G


def tt_svd(full, eps, max_rank=None):
    """TT-SVD of a dense tensor with absolute per-bond threshold ``eps``.

    Sequential truncated SVDs of the reshaped remainder (the dense
    decomposition the TT format is built from).  Returns (cores, sigmas).
    """
    full = np.asarray(full, dtype=np.float64)
    ns = full.shape
    d = len(ns)
    cores, sigmas = [], []
    rest = full.reshape(1, -1)
    r = 1
    for k in range(d - 1):
        mat = rest.reshape(r * ns[k], -1)
        U, S, Vt = np.linalg.svd(mat, full_matrices=False)
        t, _ = select_rank(S, eps, max_rank)
        sigmas.append(S)
        cores.append(U[:, :t].reshape(r, ns[k], t))
        rest = S[:t, None] * Vt[:t]
        r = t
    cores.append(rest.reshape(r, ns[d - 1], 1))
    return cores, sigmas


def compression_ratio(cores):
    """Storage in TT format over dense storage (Section 2, compression ratio)."""
    num = sum(c.size for c in cores)
    den = math.prod(c.shape[1] for c in cores)
    return num / den


def compression_gain(x, x_rounded):
    """Ratio of TT storage before and after rounding (Section 2, gain)."""
    return sum(c.size for c in x) / sum(c.size for c in x_rounded)
