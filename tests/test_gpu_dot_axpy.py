"""GPU TT inner products and TT axpy against the oracle (bit-level structure, FP tolerance)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2211_08770_amd import synth
from gpu_util import need_gpu, dev_tt, dev_sum, host_cores

pytestmark = pytest.mark.gpu


def rand(seed, ns, ranks, scale=1.0):
    return synth.random_tt(synth.rng(seed), ns, ranks, np.float64, scale)


# FP32 cores are widened exactly and every product and sum of the dot is FP64,
# so FP32 inputs meet the FP64 oracle (run on the same values upcast) at the
# FP64 level too.
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-12)])
def test_dot_pairs_and_sums(dtype, tol):
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    ns = [4, 7, 3, 5]
    xs = [[c.astype(npdt) for c in rand(10 + i, ns, [1, 2 + i, 3, 2, 1])] for i in range(3)]
    ys = [[c.astype(npdt) for c in rand(20 + i, ns, [1, 3, 1 + i, 4, 1])] for i in range(3)]
    up = lambda v: [c.astype(np.float64) for c in v]
    for x, y in zip(xs, ys):
        ref = oracle.tt_dot(up(x), up(y))
        got = tt.dot(dev_tt(x, dtype), dev_tt(y, dtype))
        assert abs(got - ref) <= tol * oracle.tt_norm(up(x)) * oracle.tt_norm(up(y))
    sx = [(0.5, xs[0]), (-2.0, xs[1])]
    sy = [(1.5, ys[2]), (1.0, ys[0]), (-1.0, ys[1])]
    ref = oracle.tt_dot(oracle.tt_sum([(a, up(v)) for a, v in sx]), oracle.tt_sum([(a, up(v)) for a, v in sy]))
    got = tt.dot(dev_sum(sx, dtype), dev_sum(sy, dtype))
    scale = sum(abs(a) * oracle.tt_norm(up(v)) for a, v in sx) * sum(abs(a) * oracle.tt_norm(up(v)) for a, v in sy)
    assert abs(got - ref) <= tol * scale
    batch = tt.dot_batched([(dev_tt(x, dtype), dev_tt(y, dtype)) for x, y in zip(xs, ys)])
    for b, x, y in zip(batch, xs, ys):
        assert abs(b - oracle.tt_dot(up(x), up(y))) <= tol * oracle.tt_norm(up(x)) * oracle.tt_norm(up(y))


def test_dot_order_one_and_rank_one_closed_form():
    tt = need_gpu()
    g = synth.rng(30)
    u = [g.standard_normal(n) for n in (5, 3, 4)]
    v = [g.standard_normal(n) for n in (5, 3, 4)]
    x = [a.reshape(1, -1, 1) for a in u]
    y = [a.reshape(1, -1, 1) for a in v]
    ref = np.prod([a @ b for a, b in zip(u, v)])
    assert abs(tt.dot(dev_tt(x), dev_tt(y)) - ref) <= 1e-13 * np.prod([np.linalg.norm(a) * np.linalg.norm(b) for a, b in zip(u, v)])
    assert abs(tt.dot(dev_tt([x[0]]), dev_tt([y[0]])) - u[0] @ v[0]) <= 1e-13 * 10


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_axpy_matches_oracle_exactly_in_structure(dtype):
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    for d in (1, 2, 4):
        ns = [3, 5, 4, 2][:d]
        x = [c.astype(npdt) for c in rand(40 + d, ns, [1] + [2] * (d - 1) + [1])]
        y = [c.astype(npdt) for c in rand(50 + d, ns, [1] + [3] * (d - 1) + [1])]
        z = tt.axpy(-1.25, dev_tt(x, dtype), dev_tt(y, dtype))
        ref = oracle.tt_axpy(-1.25, [c.astype(np.float64) for c in x], [c.astype(np.float64) for c in y])
        assert z.r == oracle.tt_ranks(ref)
        for a, b in zip(host_cores(z), ref):
            # block copies; only the first core is scaled (one multiply, rounded in the storage dtype)
            assert np.allclose(a, b, rtol=(1e-15 if dtype == torch.float64 else 1e-7), atol=0)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_norm_of_lazy_sums(dtype, tol):
    """tt_norm: right-to-left sweep then ||G_0||_F, against the oracle's orthogonalisation."""
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    up = lambda v: [c.astype(np.float64) for c in v]
    ns = [5, 6, 4, 3]
    a = [c.astype(npdt) for c in rand(41, ns, [1, 3, 4, 2, 1])]
    b = [c.astype(npdt) for c in rand(42, ns, [1, 2, 2, 3, 1])]
    # a plain TT, a sum, and a difference that nearly cancels (a - (a + 1e-6 b))
    cases = [[(1.0, a)], [(0.7, a), (-1.3, b)], [(1.0, a), (-1.0, a), (-1e-6, b)]]
    for terms in cases:
        ref_sum = oracle.tt_sum([(c, up(v)) for c, v in terms])
        ref = float(np.linalg.norm(oracle.tt_orth_rl(ref_sum)[0][0]))
        got = tt.norm(dev_sum(terms, dtype))
        scale = sum(abs(c) * oracle.tt_norm(up(v)) for c, v in terms)
        assert abs(got - ref) <= tol * scale, (got, ref)
    # order one: the plain vector norm of the summed components
    v1 = [np.arange(1.0, 8.0).reshape(1, 7, 1).astype(npdt)]
    v2 = [np.full((1, 7, 1), 0.5, dtype=npdt)]
    got = tt.norm(dev_sum([(2.0, v1), (-1.0, v2)], dtype))
    assert abs(got - np.linalg.norm(2.0 * np.arange(1.0, 8.0) - 0.5)) <= tol * 30
    # zero tensor
    z = [np.zeros((1, 4, 2)), np.zeros((2, 4, 1))]
    assert tt.norm(dev_tt([c.astype(npdt) for c in z], dtype)) == 0.0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_dot_tiles_and_split_reductions(dtype):
    """Ranks spanning several 16 x 16 matrix-core tiles with ragged edges, rank one
    against rank 40, and a long second product (r n = 33 * 64) that the kernel
    splits over waves: FP64 accumulation against the oracle in both dtypes."""
    tt = need_gpu()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    up = lambda v: [c.astype(np.float64) for c in v]
    cases = [([9, 64, 5], [1, 33, 17, 1], [1, 40, 3, 1]),
             ([16, 3, 17, 5], [1, 1, 1, 1, 1], [1, 40, 21, 6, 1]),
             ([50, 50], [1, 19, 1], [1, 47, 1])]
    for i, (ns, rx, ry) in enumerate(cases):
        x = [c.astype(npdt) for c in rand(60 + i, ns, rx)]
        y = [c.astype(npdt) for c in rand(70 + i, ns, ry)]
        ref = oracle.tt_dot(up(x), up(y))
        got = tt.dot(dev_tt(x, dtype), dev_tt(y, dtype))
        assert abs(got - ref) <= 1e-12 * oracle.tt_norm(up(x)) * oracle.tt_norm(up(y)), (ns, got, ref)
        # <x, x> is ||x||^2 to FP64 accuracy
        assert abs(tt.dot(dev_tt(x, dtype), dev_tt(x, dtype)) / oracle.tt_norm(up(x)) ** 2 - 1.0) <= 1e-12
