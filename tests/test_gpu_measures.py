"""GPU orthogonality measures against the oracle: the FP64 Gram matrix of many
TT-vectors (the Gram scheme's size at order 6: 50 generators of rank 8, n = 64,
1275 inner products), kappa(A_k) = sqrt(kappa(G_k)) against a dense SVD of the
vectorised inputs (20 vectors of order 4, cond(Gram) = 1e6), and the loss of
orthogonality of an FP32 basis at the FP64 floor (Section 3.4)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2211_08770_amd import synth
from gpu_util import need_gpu, dev_tt, dev_sum
from inputs import conditioned_inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_gram_of_fifty_order6_generators(dtype):
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    t = synth.conditioned_terms(20001, 50, 6, 64, 8, dtype=npdt)
    t64 = [[c.astype(np.float64) for c in tj] for tj in t]
    ref = oracle.gram_of(t64)
    kap, G = tt.cond([dev_tt(tj, dtype) for tj in t])
    nrm = np.sqrt(np.diag(ref))
    assert np.abs(G - ref).max() <= 1e-12 * nrm.max() ** 2
    assert np.array_equal(G, G.T)
    assert np.isfinite(kap).all() and kap[0] == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_kappa_of_conditioned_inputs_against_dense_svd(dtype):
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    X, C, M = conditioned_inputs(10000, 20, 4, 8, 3, 1e6, dtype=npdt)
    up = [[(a, [c.astype(np.float64) for c in v]) for a, v in x] for x in X]
    ref = oracle.cond_curve(up)
    kap, G = tt.cond([dev_sum(x, dtype) for x in X])
    # G_k's smallest eigenvalue carries an error of about u * ||G||; with
    # kappa(G) <= 1e6 that is a relative error of about 1e-10 in kappa(A_k)
    assert np.allclose(kap, ref, rtol=1e-8, atol=0), (kap, ref)
    assert kap[-1] == pytest.approx(1e3, rel=1e-6)


def test_loo_of_fp32_basis_at_fp64_floor():
    tt = need_gpu()
    X, C, M = conditioned_inputs(10000, 12, 4, 8, 3, 1e4, dtype=np.float32)
    Q, R, loo_run, st = tt.orthogonalize("mgs2", [dev_sum(x, torch.float32) for x in X], 1e-5)
    host = [[c.astype(np.float64) for c in q.numpy_cores()] for q in Q]
    ref = oracle.loo_curve(host)
    loo, G = tt.loo(Q)
    # the FP32 basis is orthogonal to about 1e-7; its measured loss must agree
    # with the FP64 oracle's on the same (upcast) values to rounding level
    assert np.abs(loo - ref).max() <= 1e-13, (loo, ref)
    assert np.abs(np.asarray(loo_run) - ref).max() <= 1e-13
    assert np.abs(G - oracle.gram_of(host)).max() <= 1e-13
