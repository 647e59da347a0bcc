"""TSQR tree-shape autotuner: the chosen shapes are valid, and roundings planned
with them still match the oracle (only the time depends on the shape)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2211_08770_amd import synth
from gpu_util import need_gpu, dev_tt, host_cores, diff_norm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rows,cols,dtype", [(6400, 200, torch.float32), (1500, 40, torch.float64), (300, 96, torch.float64)])
def test_tuned_shape_is_valid(rows, cols, dtype):
    tt = need_gpu()
    leaf, fanin = tt.tune_tsqr(rows, cols, dtype)
    maxrows = 800   # rows of one QR tile (the LDS panel)
    assert min(cols, rows) <= leaf <= maxrows
    assert fanin >= 2 and fanin * min(leaf, cols) <= maxrows
    if rows <= 768:
        assert leaf <= rows


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_rounding_with_autotune_matches_oracle(dtype, tol):
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    g = synth.rng(60001)
    # two summed random TTs of order 4, n = 24, rank 30: unfoldings of 720 x 60 and 24 x 60
    terms = [[c.astype(npdt) for c in synth.random_tt(g, [24] * 4, [1, 30, 30, 30, 1])] for _ in range(2)]
    x = [(1.0, dev_tt(terms[0], dtype)), (0.5, dev_tt(terms[1], dtype))]
    tt.set_autotune(True)
    try:
        out = tt.round(x, 1e-3)
    finally:
        tt.set_autotune(False)
    ref_in = oracle.tt_sum([(1.0, [c.astype(np.float64) for c in terms[0]]),
                            (0.5, [c.astype(np.float64) for c in terms[1]])])
    ref = oracle.tt_round(ref_in, 1e-3)
    assert out.r == oracle.tt_ranks(ref)
    assert diff_norm(host_cores(out), ref) <= max(tol, 1e-12) * oracle.tt_norm(ref_in)
