"""The seeded input recipes (paper_2211_08770_amd/synth.py) produce the workloads they state.

Both the oracle and the HIP path read these inputs, so a drifted recipe would change every
measured workload without failing a parity test.  Checked here: the graded sum scales term j
by 2^-j on every core; the uneven batch covers the stated ranges of order, mode size and rank;
a serving solver's right part is right-orthonormal and its first cores orthonormal, so the
norm of any solver vector is that of its first core (computed by the oracle's TT norm); the
spectrum and correlation helpers give the prescribed eigenvalues and unit diagonal.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2211_08770_amd import synth


def test_graded_sum_scales_term_j_by_2_to_minus_j_on_every_core():
    terms = synth.sum_of_graded_terms()
    assert len(terms) == 20 and all(a == 1.0 for a, _ in terms)
    for j, (_, cores) in enumerate(terms):
        assert [c.shape for c in cores] == [(1, 32, 10)] + [(10, 32, 10)] * 6 + [(10, 32, 1)]
        for c in cores:
            # i.i.d. N(0, 1) entries times 2^-j: the Frobenius norm is 2^-j sqrt(size) to a few
            # percent (relative spread about 1 / sqrt(2 size))
            expect = 2.0 ** -j * math.sqrt(c.size)
            assert abs(np.linalg.norm(c) / expect - 1.0) < 8.0 / math.sqrt(2 * c.size)
    # float32 draws are the float64 draws rounded once
    t32 = synth.sum_of_graded_terms(dtype=np.float32)
    assert all(np.array_equal(a.astype(np.float32), b) for (_, x), (_, y) in zip(terms, t32) for a, b in zip(x, y))


def test_uneven_batch_covers_the_stated_ranges():
    jobs = synth.uneven_jobs()
    assert len(jobs) == 256
    ds, ns, rs = zip(*[meta for _, meta in jobs])
    assert min(ds) == 4 and max(ds) == 10
    assert set(ns) == {16, 32, 64}
    assert 8 <= min(rs) <= 12 and 124 <= max(rs) <= 128
    for cores, (d, n, R) in jobs[:32]:
        assert len(cores) == d and all(c.dtype == np.float32 for c in cores)
        assert [c.shape for c in cores] == [(1, n, R)] + [(R, n, R)] * (d - 2) + [(R, n, 1)]
    vals = np.concatenate([c.ravel() for cores, _ in jobs[:8] for c in cores]).astype(np.float64)
    assert abs(vals.mean()) < 0.01 and abs(vals.std() - 1.0) < 0.01


def test_serving_solver_vectors_have_the_norm_of_their_first_core():
    g = synth.rng(40000)
    seen_d, seen_n = set(), set()
    for _ in range(12):
        s = synth.serving_solver(g, dtype=np.float64)
        d, n, r = s["d"], s["n"], s["r"]
        seen_d.add(d)
        seen_n.add(n)
        assert 5 <= d <= 8 and n in (32, 64, 128) and 4 <= r <= 32 and 10 <= s["b0"] <= 39
        for c in s["right"]:   # right-orthonormal: rows of the right unfolding orthonormal
            U = c.reshape(c.shape[0], -1)
            assert np.allclose(U @ U.T, np.eye(c.shape[0]), atol=1e-12)
        F = np.stack([f.ravel() for f in s["firsts"]], axis=1)
        assert F.shape == (n * r, 40) and np.allclose(F.T @ F, np.eye(40), atol=1e-12)
        w = synth.serving_request(g, s, s["b0"])
        assert w.shape == (1, n, r)
        for first in (s["firsts"][0], w):
            v = synth.serving_vector(g, s, first)
            assert abs(oracle.tt_norm(v) - np.linalg.norm(first)) <= 1e-12 * np.linalg.norm(first)
    assert len(seen_d) >= 3 and len(seen_n) >= 2


@pytest.mark.parametrize("m,kappa", [(6, 1e6), (20, 1e6), (50, 1e10)])
def test_spectrum_and_correlation_helpers(m, kappa):
    lam = synth.geometric_spectrum(m, kappa)
    assert lam.sum() == pytest.approx(m) and lam.max() / lam.min() == pytest.approx(kappa, rel=1e-9)
    M = synth.correlation_with_spectrum(7, lam)
    assert np.allclose(np.diag(M), 1.0, atol=1e-12)
    ev = np.sort(np.linalg.eigvalsh(M))
    assert np.allclose(ev, np.sort(lam), rtol=1e-6, atol=1e-12 * m)
