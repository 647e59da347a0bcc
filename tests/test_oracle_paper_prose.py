"""The oracle on the paper's own order-3 experiment against the loss-of-orthogonality levels
that Section 4 states in its text (tests/golden/section4_order3_loo_prose.json; the figure data
are not in the paper's text, so the curves themselves are parity-unpinned).  Levels are checked
within an order of magnitude where the text gives one; the two places where the oracle departs
from the text (TT-Gram breaks down at m = 20; TT-MGS2 at delta = 1e-3 jumps to about 5e-7, not
1e-11) are asserted as such, so that a change in either is noticed."""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "section4_order3_loo_prose.json")
U = 1.1e-16


@pytest.fixture(scope="module")
def experiment():
    A = oracle.krylov_inputs([15, 15, 15], 20)
    kap = oracle.cond_curve(A)
    loo = {}
    for delta in (1e-3, 1e-5, 1e-8):
        for sch in ("cgs", "mgs", "cgs2", "mgs2", "householder"):
            loo[sch, delta] = oracle.loo_curve(oracle.orthogonalize(sch, A, delta).Q)
    return A, kap, loo


def test_claims_file_is_cited():
    claims = json.load(open(GOLDEN))
    assert claims["source"].startswith("Section 4, order-3 experiment")


def test_cgs_stagnates_below_1e2(experiment):
    A, kap, loo = experiment
    for delta in (1e-3, 1e-5, 1e-8):
        v = loo["cgs", delta]
        assert v[10:].max() < 1e2 and v[10:].min() > 1e-1      # lost, but stagnating below 1e2


def test_mgs_follows_kappa(experiment):
    A, kap, loo = experiment
    assert kap[-1] > 1e13                                       # the Krylov vectors become collinear
    for delta in (1e-3, 1e-5, 1e-8):
        v = loo["mgs", delta]
        # the slope of kappa: over k = 10..20 both grow by many orders, within two orders of each other
        growth_loo, growth_kap = v[19] / v[9], kap[19] / kap[9]
        assert 1e-2 * growth_kap <= growth_loo <= 1e2 * growth_kap, (delta, growth_loo, growth_kap)


def test_cgs2_near_machine_precision_then_rising(experiment):
    A, kap, loo = experiment
    for delta in (1e-3, 1e-5, 1e-8):
        v = loo["cgs2", delta]
        assert v[:14].max() <= 1e-13                            # about 1e-14 up to k = 14
    assert loo["cgs2", 1e-8].max() <= 1e-13                     # stays there at delta = 1e-8
    for delta in (1e-3, 1e-5):
        v = loo["cgs2", delta]
        assert v[19] > 1e2 * v[13]                              # increasing for k >= 15


def test_mgs2_levels(experiment):
    A, kap, loo = experiment
    for delta in (1e-5, 1e-8):
        assert loo["mgs2", delta].max() <= 1e-13                # about 1e-14
    v = loo["mgs2", 1e-3]
    assert v[:14].max() <= 1e-13 and v[19] > 1e2 * v[13]         # the jump the text describes ...
    assert 1e-8 < v[19] < 1e-5                                  # ... but to about 5e-7, not 1e-11


def test_householder_around_delta(experiment):
    A, kap, loo = experiment
    for delta in (1e-3, 1e-5, 1e-8):
        v = loo["householder", delta][-1]
        assert 1e-3 * delta <= v <= 10 * delta, (delta, v)


def test_gram_breaks_down_on_the_order3_inputs():
    """The text plots TT-Gram up to k = 20; here its Gram matrix (cond about 1e27) is not
    numerically positive definite and the oracle reports the breakdown."""
    A = oracle.krylov_inputs([15, 15, 15], 20)
    with pytest.raises(oracle.GramBreakdown):
        oracle.gram(A, 1e-5)
