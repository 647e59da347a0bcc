"""Host logic of the binding: the output-capacity bounds of tt.orthogonalize cover the ranks
that every scheme actually produces (checked against the oracle's q_i; no GPU needed)."""
import pytest

import oracle
from inputs import conditioned_inputs
from paper_2211_08770_amd.tt import q_rank_bounds


@pytest.mark.parametrize("scheme", ["cgs", "mgs", "cgs2", "mgs2", "gram", "householder"])
@pytest.mark.parametrize("delta", [1e-3, 1e-10])
def test_q_rank_bounds_cover_the_oracle_ranks(scheme, delta):
    X, _, _ = conditioned_inputs(700, 6, 3, 4, 2, 1e3)
    ns = [4, 4, 4]
    ra = []
    for s in X:
        r = [0] * 4
        for _, cores in s:
            for k, kr in enumerate(oracle.tt_ranks(cores)):
                r[k] += kr
        ra.append(r)
    bounds = q_rank_bounds(scheme, ra, ns)
    res = oracle.orthogonalize(scheme, X, delta)
    for q, b in zip(res.Q, bounds):
        assert all(a <= c for a, c in zip(oracle.tt_ranks(q), b)), (scheme, oracle.tt_ranks(q), b)


def test_q_rank_bounds_respect_caps_and_guard():
    ra = [[1, 5, 5, 1]] * 4
    for scheme in ("cgs", "gram", "householder"):
        for b in q_rank_bounds(scheme, ra, [3, 3, 3], rank_guard=0):
            assert b[0] == b[-1] == 1 and b[1] <= 3 and b[2] <= 3
        for b in q_rank_bounds(scheme, [[1, 50, 50, 1]] * 4, [10, 10, 10], rank_guard=7):
            assert max(b) <= 7
