"""Pins for the oracle's window bounds (chi-square quantiles, paper weights).

The bound of a window S is the chi-square(|S|) 0.9 quantile; the paper's own
weights (Sec. 2.1) are c_s = (q sigma_s + mu_s)^-4, i.e. bound 1/c_s.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

import oracle


@pytest.mark.parametrize("k", [1, 2, 3, 4, 9, 16, 25, 64, 81, 100, 144, 225, 256, 1024])
@pytest.mark.parametrize("p", [0.5, 0.9, 0.99])
def test_quantile_matches_scipy(k, p):
    got = oracle.chi2_quantile(k, p)
    ref = stats.chi2.ppf(p, k)
    assert abs(got - ref) <= 1e-12 * ref


def test_closed_forms():
    # 1 dof: the square of the two-sided normal quantile.
    z = special.ndtri(0.95)
    assert oracle.chi2_quantile(1, 0.9) == pytest.approx(z * z, rel=1e-13)
    # 2 dof: exponential law with mean 2, quantile -2 ln(1-p).
    for p in (0.1, 0.5, 0.9, 0.999):
        assert oracle.chi2_quantile(2, p) == pytest.approx(-2.0 * math.log1p(-p), rel=1e-13)


@pytest.mark.parametrize("k", [1, 2, 5, 16, 81, 256])
def test_cdf_matches_regularised_gamma(k):
    for x in (0.3, 1.0, k * 0.7, k * 1.0, k * 1.6 + 3):
        assert oracle.chi2_cdf(k, x) == pytest.approx(special.gammainc(k / 2.0, x / 2.0),
                                                       rel=1e-12, abs=1e-15)


def test_bounds_for_window_sides():
    sides = list(range(1, 17))
    r2 = oracle.chi2_bounds(sides)
    assert np.all(np.diff(r2) > 0)
    # Known values, 0.9 quantile: s=1 -> 2.70554..., s=2 (4 dof) -> 7.77944...
    assert r2[0] == pytest.approx(2.705543454095404, rel=1e-14)
    assert r2[1] == pytest.approx(7.779440339734858, rel=1e-14)


def test_paper_bound_closed_forms():
    # q_alpha = 0: bound = mu^4 = n - 1/2 exactly.
    for n in (1, 4, 9, 64, 256):
        assert oracle.paper_bound(n, 0.0) == pytest.approx(n - 0.5, rel=1e-14)
    # Derivative in q at 0 is 4 mu^3 sigma with sigma^2 = 1/(8 sqrt n).
    n, h = 16, 1e-6
    d = (oracle.paper_bound(n, h) - oracle.paper_bound(n, -h)) / (2 * h)
    mu = (n - 0.5) ** 0.25
    assert d == pytest.approx(4 * mu ** 3 / math.sqrt(8 * math.sqrt(n)), rel=1e-7)
