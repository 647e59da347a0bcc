"""Serving engine (continuous batching of Gram-Schmidt steps).

A request is exactly the step i = b of the scheme (Algorithms 1-4) run by
tt_orthogonalize on the same inputs; a request's result is the same alone
and in a mix of concurrent requests that join at different times; the
serving loop completes a Poisson trace and keeps the bases orthonormal.
"""
import numpy as np
import pytest
import torch

from paper_2211_08770_amd import synth
from gpu_util import need_gpu, dev_sum
from inputs import conditioned_inputs

pytestmark = pytest.mark.gpu


def _run_alone(eng, *args, **kw):
    rid = eng.submit(*args, **kw)
    for _ in range(50):
        out = eng.step()
        if rid in out:
            return out[rid]
    raise AssertionError("request did not complete")


@pytest.mark.parametrize("scheme", ["mgs2", "cgs2", "mgs", "cgs"])
def test_engine_request_equals_scheme_step(scheme):
    tt = need_gpu()
    X, _, _ = conditioned_inputs(50001, 6, 4, 5, 2, 1e3)
    A = [dev_sum(x) for x in X]
    Q, R, _, _ = tt.orthogonalize(scheme, A, 1e-10)
    b = 5
    _, G = tt.loo(Q[:b])
    eng = tt.Engine()
    status, q, r, grow = _run_alone(eng, scheme, Q[:b], A[b], 1e-10, basis_gram=G)
    assert status == "TT_OK"
    assert q.r == Q[b].r
    assert torch.equal(q.data, Q[b].data)
    assert np.array_equal(r, R[: b + 1, b])
    _, G6 = tt.loo(Q[:b] + [q])
    assert np.allclose(grow, G6[b, :b], rtol=0, atol=1e-15)


def _small_solvers(tt, seed, count, dtype):
    from paper_2211_08770_amd import serve
    return serve.make_solvers(count, seed=seed, dtype=dtype, d_range=(3, 4), n_choices=(6, 8), r_range=(2, 3),
                              b0_range=(3, 5), bmax=8)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_result_is_the_same_alone_and_in_a_mix(dtype):
    tt = need_gpu()
    solvers, g = _small_solvers(tt, 40101, 4, dtype)

    def request(s, seed):
        gg = synth.rng(seed)
        w = synth.serving_request(gg, s.spec, len(s.basis))
        return tt.TT.from_cores(synth.serving_vector(None, s.spec, w), device="cuda", dtype=dtype)

    x_solver = solvers[0]
    wx = request(x_solver, 7)
    eng = tt.Engine()
    alone = _run_alone(eng, "mgs2", x_solver.basis, wx, 1e-6, basis_gram=x_solver.gram)
    assert alone[0] == "TT_OK"
    # the mix: two requests start first, X joins two steps later, a fourth joins after X
    ids = [eng.submit("mgs2", solvers[1].basis, request(solvers[1], 8), 1e-6, basis_gram=solvers[1].gram),
           eng.submit("cgs2", solvers[2].basis, request(solvers[2], 9), 1e-6)]
    results = {}
    for _ in range(2):
        results.update(eng.step())
    rx = eng.submit("mgs2", x_solver.basis, wx, 1e-6, basis_gram=x_solver.gram)
    results.update(eng.step())
    ids.append(eng.submit("mgs", solvers[3].basis, request(solvers[3], 10), 1e-6, basis_gram=solvers[3].gram))
    for _ in range(20):
        results.update(eng.step())
        if all(i in results for i in ids + [rx]):
            break
    assert all(results[i][0] == "TT_OK" for i in ids + [rx])
    mixed = results[rx]
    assert mixed[1].r == alone[1].r
    assert torch.equal(mixed[1].data, alone[1].data)
    assert np.array_equal(mixed[2], alone[2]) and np.array_equal(mixed[3], alone[3])
    assert eng.pending() == 0


def test_breakdown_on_a_zero_vector():
    tt = need_gpu()
    solvers, _ = _small_solvers(tt, 40201, 1, torch.float64)
    s = solvers[0]
    zero = tt.TT.from_cores(synth.serving_vector(None, s.spec, np.zeros((1, s.spec["n"], s.spec["r"]))),
                            device="cuda", dtype=torch.float64)
    eng = tt.Engine()
    status, _, r, _ = _run_alone(eng, "mgs2", s.basis, zero, 1e-8, basis_gram=s.gram)
    assert status == "TT_EBREAKDOWN" and r[-1] == 0.0


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
def test_serving_trace_keeps_bases_orthonormal(dtype, tol):
    tt = need_gpu()
    from paper_2211_08770_amd import serve
    solvers, g = _small_solvers(tt, 40301, 6, dtype)
    b_before = [len(s.basis) for s in solvers]
    rep = serve.run_trace(solvers, g, qps=2000.0, nreq=24, delta=1e-8 if dtype == torch.float64 else 1e-5,
                          max_inflight=6)
    assert rep["completed"] == 24 and rep["rejected"] == 0
    assert rep["p50_ms"] > 0 and rep["p99_ms"] >= rep["p50_ms"]
    grown = sum(len(s.basis) for s in solvers) - sum(b_before)
    assert grown > 0
    for s in solvers:
        loo, _ = tt.loo(s.basis)
        assert loo[-1] <= tol * len(s.basis), (loo[-1], len(s.basis))
        # every basis vector keeps the solver's rank (the rounding compresses the projections back)
        assert all(max(q.r) <= s.spec["r"] for q in s.basis)


def test_fp32_requests_at_stated_workload_against_oracle_step():
    """MGS2 requests of the serving workload (solvers with d ~ U{5..8}, n ~ U{32,64,128},
    rank ~ U{4..9}, 10-39 resident basis vectors; FP32-bulk, delta = 1e-6) against the
    oracle's MGS2 step on the same FP32 values upcast: q by difference norm and the R
    column within max(delta, 1e-5) (the basis is orthonormal and w well separated from
    its span, so kappa is about one)."""
    tt = need_gpu()
    import oracle
    from gpu_util import host_cores, diff_norm
    from paper_2211_08770_amd import serve
    solvers, g = serve.make_solvers(3, seed=40401, dtype=torch.float32)
    eng = tt.Engine()
    for k, s in enumerate(solvers):
        first = synth.serving_request(synth.rng(41000 + k), s.spec, len(s.basis))
        wc = synth.serving_vector(None, s.spec, first)
        w = tt.TT.from_cores(wc, device="cuda", dtype=torch.float32)
        status, q, r, _ = _run_alone(eng, "mgs2", s.basis, w, 1e-6, basis_gram=s.gram)
        assert status == "TT_OK"
        basis64 = [host_cores(b) for b in s.basis]
        qref, cref = oracle.gs_step("mgs2", basis64, [c.astype(np.float64) for c in wc], 1e-6)
        nw = oracle.tt_norm([c.astype(np.float64) for c in wc])
        assert np.abs(r - cref).max() <= 1e-5 * nw, (k, s.spec["d"], s.spec["n"], np.abs(r - cref).max())
        assert diff_norm(host_cores(q), qref) <= 1e-5, (k, diff_norm(host_cores(q), qref))
