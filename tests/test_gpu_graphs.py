"""Graph replay of bound-planned batched roundings (tt_ctx_set_graphs + tt_round_batched_async):
the first run is captured, later runs launch the graph.  Every replay is checked against the
eager (uncaptured) rounding of the same data, with the program's own eager work and
synchronisations between the replays, and one job against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2211_08770_amd import synth
from gpu_util import need_gpu, dev_tt, host_cores, diff_norm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_replays_equal_eager_roundings(dtype):
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    jobs = synth.uneven_jobs(seed=30031, njobs=9, d_range=(2, 6), n_choices=(3, 4, 8), r_range=(2, 16),
                             dtype=npdt)
    graded = synth.sum_of_graded_terms(nterms=5, d=4, n=6, r=3, dtype=npdt)
    xs = [dev_tt(c, dtype) for c, _ in jobs] + [[(a, dev_tt(t, dtype)) for a, t in graded]]
    delta = 1e-6
    br = tt.BatchRounder(xs, delta)
    bufs = [x.data for x in xs[:-1]] + [t.data for _, t in xs[-1]]
    for it in range(4):
        if it:
            # new data in the same buffers: every replay must see it
            for b in bufs:
                b.mul_(1.0 + 0.25 * it)
            torch.cuda.synchronize()
        br.run()
        got = br.results()
        assert br.graph_count() == 1
        eager = tt.round_batched(xs, delta, plan="bounds")
        for g, e in zip(got, eager):
            assert g.r == e.r and torch.equal(g.data, e.data), it
        # some unrelated eager work and a synchronisation between the replays
        other = tt.round(xs[0], 1e-3)
        torch.cuda.synchronize()
        assert other.r[0] == 1
    # the graded sum (ranks below their bounds: the compaction moves cores) against the oracle
    x64 = oracle.tt_sum([(a, host_cores(t)) for a, t in xs[-1]])   # the data the last replay saw
    ref = oracle.tt_round(x64, delta)
    assert got[-1].r == oracle.tt_ranks(ref)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert diff_norm(host_cores(got[-1]), ref) <= tol * oracle.tt_norm(x64)
