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


@pytest.mark.parametrize("scheme", ["cgs2", "mgs2"])
@pytest.mark.parametrize("delta", [0.0, 1e-12])
def test_two_pass_bounds_where_the_caps_do_not_bind(scheme, delta):
    """Mode sizes large enough that no rank cap binds: the second pass rounds the
    first pass's result (up to rank(a_i) + sum of earlier q ranks) plus the basis
    again, and at delta = 0 the rounding keeps every nonzero singular value, so
    the q ranks reach that sum; the bounds must cover it."""
    X, _, _ = conditioned_inputs(710, 4, 3, 30, 2, 1e2)
    ns = [30, 30, 30]
    ra = [[sum(oracle.tt_ranks(c)[k] for _, c in s) for k in range(4)] for s in X]
    bounds = q_rank_bounds(scheme, ra, ns)
    res = oracle.orthogonalize(scheme, X, delta)
    for q, b in zip(res.Q, bounds):
        assert all(a <= c for a, c in zip(oracle.tt_ranks(q), b)), (scheme, oracle.tt_ranks(q), b)
    # the second pass really exceeds the first-pass sum here
    assert any(oracle.tt_ranks(q)[1] > r[1] + sum(oracle.tt_ranks(p)[1] for p in res.Q[:i])
               for i, (q, r) in enumerate(zip(res.Q, ra))) or delta > 0


def test_capacity_query_sizes_and_errors():
    """tt_orthogonalize_capacity: packed sizes agree with the rank bounds; bad shapes are rejected."""
    import ctypes as C
    from paper_2211_08770_amd import tt
    lib = tt._load()
    ns = [4, 5, 6]
    ra = [[1, 3, 3, 1], [1, 4, 2, 1]]
    b = q_rank_bounds("mgs", ra, ns)
    assert b[0] == [1, 3, 3, 1] and b[1] == [1, 4, 5, 1]   # 4+3 capped by 4; 2+3 = 5 <= 6
    with pytest.raises(tt.TTError):
        q_rank_bounds("cgs", [[1, 0, 3, 1]], ns)          # ranks must be >= 1
