"""Helpers of the GPU parity tests: moving TTs to the device and comparing
results with the oracle by reconstruction (never by cores)."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_08770_amd import tt
    tt._load()          # raises when the HIP library is missing: no silent fallback
    return tt


def dev_tt(cores, dtype=torch.float64):
    from paper_2211_08770_amd.tt import TT
    return TT.from_cores([np.ascontiguousarray(c) for c in cores], device="cuda", dtype=dtype)


def dev_sum(terms, dtype=torch.float64):
    return [(float(a), dev_tt(x, dtype)) for a, x in terms]


def host_cores(t):
    return [c.astype(np.float64) for c in t.numpy_cores()]


def diff_norm(a, b):
    """||a - b|| for two TTs, by a TT difference and an orthogonalisation sweep."""
    s = oracle.tt_sum([(1.0, a), (-1.0, b)])
    G, _ = oracle.tt_orth_rl(s)
    return float(np.linalg.norm(G[0]))


def left_orth_error(cores):
    err = 0.0
    for c in cores[:-1]:
        r0, n, r1 = c.shape
        L = c.reshape(r0 * n, r1)
        err = max(err, float(np.abs(L.T @ L - np.eye(r1)).max()))
    return err


def sample_entries(cores, idx):
    out = []
    for ix in idx:
        m = np.ones((1, 1))
        for k, i in enumerate(ix):
            m = m @ cores[k][:, i, :]
        out.append(m[0, 0])
    return np.array(out)


def rand_index(ns, count, seed=0):
    g = np.random.Generator(np.random.PCG64(seed))
    return [tuple(int(g.integers(0, n)) for n in ns) for _ in range(count)]


def min_margin(log):
    return min(log.margins) if log.margins else math.inf
