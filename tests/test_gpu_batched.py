"""Batched uneven roundings: each job equals its oracle result and is bitwise
identical to the same job rounded alone (tile choices depend only on the job)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2211_08770_amd import synth
from gpu_util import need_gpu, dev_tt, host_cores, diff_norm

pytestmark = pytest.mark.gpu


def small_uneven_jobs(seed, njobs):
    return synth.uneven_jobs(seed=seed, njobs=njobs, d_range=(2, 6), n_choices=(3, 4, 8), r_range=(2, 20),
                             dtype=np.float64)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_uneven_matches_oracle_and_singles(dtype):
    tt = need_gpu()
    delta = 1e-5
    jobs = small_uneven_jobs(30001, 12)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    cores = [[c.astype(npdt) for c in j[0]] for j in jobs]
    xs = [dev_tt(c, dtype) for c in cores]
    outs = tt.round_batched(xs, delta)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for c, o, x in zip(cores, outs, xs):
        c64 = [a.astype(np.float64) for a in c]
        ref = oracle.tt_round(c64, delta)
        nx = oracle.tt_norm(c64)
        assert o.r == oracle.tt_ranks(ref)
        assert diff_norm(host_cores(o), ref) <= tol * nx
        single = tt.round(x, delta)
        assert single.r == o.r and torch.equal(single.data, o.data)


def test_batched_mixed_orders_including_order_one():
    """Jobs of order 1 to 4 in one batch (the norms of every job come back in one array): each
    equals its oracle result and the same job rounded alone."""
    tt = need_gpu()
    delta = 1e-6
    jobs = synth.uneven_jobs(seed=30011, njobs=10, d_range=(1, 4), n_choices=(3, 5), r_range=(1, 6),
                             dtype=np.float64)
    assert any(d == 1 for _, (d, _, _) in jobs) and any(d >= 3 for _, (d, _, _) in jobs)
    xs = [dev_tt(c, torch.float64) for c, _ in jobs]
    outs = tt.round_batched(xs, delta)
    for (c, _), o, x in zip(jobs, outs, xs):
        ref = oracle.tt_round(c, delta)
        assert o.r == oracle.tt_ranks(ref)
        assert diff_norm(host_cores(o), ref) <= 1e-12 * oracle.tt_norm(c)
        single = tt.round(x, delta)
        assert single.r == o.r and torch.equal(single.data, o.data)


def test_full_size_uneven_batch_sampled_against_oracle():
    """The 256-job uneven workload (d ~ U{4..10}, n ~ U{16,32,64}, rank ~ U{8..128}, FP32
    cores, delta = 1e-5) rounded in one batch; 16 jobs sampled across the batch (every
    16th, plus the job of largest work) each compared with the oracle's rounding of the
    same FP32 values upcast: ranks equal (the caps; there is no compressible tail) and
    error within max(delta, 1e-5)."""
    tt = need_gpu()
    delta = 1e-5
    jobs = synth.uneven_jobs(seed=30000)
    xs = [dev_tt(c, torch.float32) for c, _ in jobs]
    outs = tt.round_batched(xs, delta)
    # planned at the rank bounds (no host synchronisation until the end): the ranks equal the
    # bounds here, so the results are bitwise those of the host-planned batch
    bnd = tt.round_batched(xs, delta, plan="bounds")
    assert all(a.r == b.r and torch.equal(a.data, b.data) for a, b in zip(outs, bnd))
    work = [d * n * R ** 3 for _, (d, n, R) in jobs]
    pick = sorted(set(list(range(0, len(jobs), 16)) + [int(np.argmax(work))]))
    assert len(pick) >= 16
    for i in pick:
        c64 = [a.astype(np.float64) for a in jobs[i][0]]
        ref = oracle.tt_round(c64, delta)
        assert outs[i].r == oracle.tt_ranks(ref), (i, jobs[i][1])
        assert diff_norm(host_cores(outs[i]), ref) <= 1e-5 * oracle.tt_norm(c64), (i, jobs[i][1])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_planning_at_rank_bounds_matches_host_planning(dtype):
    """tt_round_batched_async (every left-to-right step planned at the rank bounds, the cores
    compacted on the device, one read-back at the end): bitwise the host-planned result for
    jobs whose ranks reach the bounds; for truncated jobs (graded sums: ranks far below the
    bounds) the same ranks and the oracle's result within the tolerance."""
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    jobs = small_uneven_jobs(30021, 10)
    cores = [[c.astype(npdt) for c in j[0]] for j in jobs]
    graded = [synth.sum_of_graded_terms(nterms=6, d=d, n=n, r=4, dtype=npdt) for d, n in ((4, 6), (5, 4), (3, 9))]
    xs = [dev_tt(c, dtype) for c in cores] + [[(a, dev_tt(t, dtype)) for a, t in g] for g in graded]
    delta = 1e-5
    host = tt.round_batched(xs, delta)
    bnd = tt.round_batched(xs, delta, plan="bounds")
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for i, (h, b) in enumerate(zip(host, bnd)):
        assert h.r == b.r, (i, h.r, b.r)
        if i < len(cores):
            c64 = [a.astype(np.float64) for a in cores[i]]
            caps = oracle.tt_ranks(oracle.tt_round(c64, 0.0))
            if h.r == caps:
                assert torch.equal(h.data, b.data), i
            x64 = c64
        else:
            x64 = oracle.tt_sum([(a, [c.astype(np.float64) for c in t]) for a, t in graded[i - len(cores)]])
        ref = oracle.tt_round(x64, delta)
        assert b.r == oracle.tt_ranks(ref)
        assert diff_norm(host_cores(b), ref) <= tol * oracle.tt_norm(x64), i
    assert any(max(b.r) < max(oracle.tt_ranks(oracle.tt_round(oracle.tt_sum(
        [(a, [c.astype(np.float64) for c in t]) for a, t in g]), 0.0))) for b, g in zip(bnd[len(cores):], graded))
