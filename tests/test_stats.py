"""Host-side statistics (no GPU): interval formulas against independent
references and their defining properties."""
from __future__ import annotations

import math

import numpy as np
import pytest
from scipy import stats as sst

from paper_2512_23037_amd.stats import bayes_factor_interval, rates, wilson


@pytest.mark.parametrize("k,n", [(0, 10), (1, 10), (5, 10), (10, 10), (3, 1000), (17, 123456), (0, 10**9)])
def test_wilson_matches_scipy(k, n):
    ci = sst.binomtest(k, n).proportion_ci(confidence_level=0.95, method="wilson")
    lo, hi = wilson(k, n)
    assert abs(lo - ci.low) < 1e-12 and abs(hi - ci.high) < 1e-12


@pytest.mark.parametrize("k,n", [(1, 10), (5, 10), (3, 1000), (17, 123456), (400, 10**7)])
def test_bayes_interval_endpoints_have_the_likelihood_ratio(k, n):
    lo, hi = bayes_factor_interval(k, n)
    ph = k / n
    assert lo < ph < hi
    ll = lambda p: k * math.log(p) + (n - k) * math.log1p(-p)
    for end in (lo, hi):
        assert abs((ll(ph) - ll(end)) - math.log(1000.0)) < 1e-7
    # a wider factor gives a wider interval
    lo2, hi2 = bayes_factor_interval(k, n, factor=1e6)
    assert lo2 < lo and hi2 > hi


def test_bayes_interval_zero_successes_closed_form():
    # k = 0: L(p) = (1-p)^n, so hi = 1 - 1000^(-1/n), lo = 0
    for n in (1, 10, 1000, 10**8):
        lo, hi = bayes_factor_interval(0, n)
        assert lo == 0.0
        assert abs(hi - (1.0 - 1000.0 ** (-1.0 / n))) < 1e-12 * max(1.0, hi) + 1e-15
    lo, hi = bayes_factor_interval(7, 7)
    assert hi == 1.0 and abs(lo - 1000.0 ** (-1.0 / 7)) < 1e-12


def test_bayes_interval_normal_limit():
    # large n: the interval tends to p_hat +- sqrt(2 ln 1000) sigma
    k, n = 10**6, 10**8
    lo, hi = bayes_factor_interval(k, n)
    s = math.sqrt(k / n * (1 - k / n) / n)
    w = math.sqrt(2 * math.log(1000.0))
    assert abs((hi - lo) / (2 * w * s) - 1.0) < 1e-3


def test_rates_from_counters():
    c = {"shots": 1000, "passed": 200, "discarded": 800, "overflow": 0, "numeric": 0, "logical_errors": 2}
    r = rates(c)
    assert r["ler"] == 0.01 and r["discard_rate"] == 0.8
    assert r["ler_wilson95"][0] < 0.01 < r["ler_wilson95"][1]
