"""Pins of the oracle's Monte-Carlo weight estimation (Sec. 2.1, selection of the
weights): the field generator, the statistic Q and its quantile.

What fixes each routine independently of itself:
  * Philox4x64-10 against numpy's own implementation of the same published
    generator (numpy.random.Philox);
  * the fields against the normal law (moments, Kolmogorov-Smirnov) and the
    chi-square law of a window's sum of squares;
  * Q against a vectorised brute force over every window (numpy), and, for a
    single window, against the paper's bound formula, which inverts it;
  * the quantile against numpy's inverted-CDF quantile;
  * the defining property of the weights: with r2_s = (q sigma_s + mu_s)^4 the
    fraction of fields meeting every window bound is exactly ceil(alpha n)/n on
    the sample and about alpha on fresh fields;
  * planted mistakes in each routine are caught by these pins.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest
from numpy.lib.stride_tricks import sliding_window_view
from scipy import special, stats

import oracle
import smre_inputs as gi


def _numpy_philox_block(ctr, key):
    """numpy advances the counter before it generates, so the block of counter
    c is the first output of a generator started at c - 1 (with borrow)."""
    c = [int(v) for v in ctr]
    for i in range(4):
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = 2**64 - 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(c, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [0, 0]),
    ([5, 17, 0, 0], [12345, 0]),
    ([0, 1, 0, 0], [2**64 - 1, 0]),           # crosses a borrow in the helper
    ([2**63 + 7, 3, 9, 2**40], [0xDEADBEEF, 0xFEEDFACE]),
    ([2**64 - 1] * 4, [2**64 - 1, 2**64 - 1]),
])
def test_philox_matches_numpy(ctr, key):
    ours = oracle.philox4x64_10(ctr, key)
    ref = _numpy_philox_block(ctr, key)
    assert [int(v) for v in ours] == [int(v) for v in ref]


def test_fields_are_standard_normal():
    z = np.concatenate([oracle.mc_field(11, f, 128, 256).ravel() for f in range(4)])
    n = z.size
    assert abs(z.mean()) < 5.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # both Box-Muller outputs (cosine and sine lanes) are N(0,1) on their own
    for lane in range(4):
        zl = z[lane::4]
        assert abs(zl.var() - 1.0) < 6.0 * math.sqrt(2.0 / zl.size)
    # neighbours and fields are uncorrelated
    f0 = oracle.mc_field(11, 0, 128, 256)
    f1 = oracle.mc_field(11, 1, 128, 256)
    assert abs(np.corrcoef(f0[:, :-1].ravel(), f0[:, 1:].ravel())[0, 1]) < 0.02
    assert abs(np.corrcoef(f0.ravel(), f1.ravel())[0, 1]) < 0.02


def test_window_sums_are_chi_square():
    # the sum of squares over one 3 x 3 window, over many fields, has 9 dof
    t = np.array([np.sum(oracle.mc_field(5, f, 3, 3) ** 2) for f in range(4000)])
    assert stats.kstest(t, stats.chi2(9).cdf).pvalue > 1e-3


def test_field_depends_on_pixel_index_only():
    # pixel p = i W + j: the row-major prefix does not depend on the shape
    a = oracle.mc_field(3, 2, 4, 10).ravel()
    b = oracle.mc_field(3, 2, 10, 4).ravel()
    assert np.array_equal(a, b)
    assert not np.array_equal(oracle.mc_field(3, 2, 4, 10), oracle.mc_field(3, 3, 4, 10))
    assert not np.array_equal(oracle.mc_field(3, 2, 4, 10), oracle.mc_field(4, 2, 4, 10))


def _paper_mu_sigma(s):
    n = s * s
    return (n - 0.5) ** 0.25, math.sqrt(1.0 / (8.0 * math.sqrt(n)))


def _brute_statistic(e, sides):
    Q, tmax = -np.inf, []
    for s in sides:
        t = sliding_window_view(e * e, (s, s)).sum(axis=(2, 3))
        mu, sg = _paper_mu_sigma(s)
        Q = max(Q, float(((t ** 0.25 - mu) / sg).max()))
        tmax.append(float(t.max()))
    return Q, np.array(tmax)


@pytest.mark.parametrize("H,W,sides", [(9, 13, [1, 2, 3]), (20, 17, [1, 4, 5, 16]),
                                       (8, 8, [8]), (31, 6, [2, 6])])
def test_statistic_matches_brute_force(H, W, sides):
    e = gi.gaussian(H, W, seed=H * W)
    q, tmax = oracle.mc_statistic(e, sides)
    qb, tb = _brute_statistic(e, sides)
    assert q == pytest.approx(qb, rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(tmax, tb, rtol=1e-12)


@pytest.mark.parametrize("s", [1, 2, 3, 5, 8])
def test_single_window_statistic_inverts_paper_bound(s):
    # one window: r2 = (Q sigma + mu)^4 gives back its own sum of squares
    for seed in range(5):
        e = gi.gaussian(s, s, seed=seed)
        q, tmax = oracle.mc_statistic(e, [s])
        assert tmax[0] == pytest.approx(np.sum(e * e), rel=1e-13)
        assert oracle.paper_bound(s * s, q) == pytest.approx(tmax[0], rel=1e-11)


@pytest.mark.parametrize("s", [2, 3, 4, 8, 16])
def test_fourth_root_moments(s):
    # mu_s and sigma_s approximate the exact mean and spread of t^(1/4) for
    # t ~ chi-square(k = s^2), E t^a = 2^a Gamma(k/2 + a) / Gamma(k/2), up to
    # the second-order terms of the expansion of t^(1/4) about k: the mean is
    # off by about 1/(16 k) relative, the spread by about 1.4/(16 k)
    k = s * s
    m1 = 2 ** 0.25 * math.exp(special.gammaln(k / 2 + 0.25) - special.gammaln(k / 2))
    m2 = 2 ** 0.5 * math.exp(special.gammaln(k / 2 + 0.5) - special.gammaln(k / 2))
    sd = math.sqrt(m2 - m1 * m1)
    mu = oracle.paper_bound(k, 0.0) ** 0.25
    sg = oracle.paper_bound(k, 1.0) ** 0.25 - mu
    assert abs(mu / m1 - 1) < 1.25 / (16 * k)
    assert abs(sg / sd - 1) < 1.75 / (16 * k)


@pytest.mark.parametrize("n", [1, 2, 7, 100, 101])
@pytest.mark.parametrize("alpha", [0.01, 0.5, 0.9, 0.95, 1.0])
def test_order_quantile_matches_numpy(n, alpha):
    rng = np.random.default_rng(n)
    q = np.round(rng.standard_normal(n), 1)   # ties included
    assert oracle.order_quantile(q, alpha) == np.quantile(q, alpha, method="inverted_cdf")
    assert math.isnan(oracle.order_quantile(q, 0.0))
    assert math.isnan(oracle.order_quantile(q, 1.5))


def _sample(seed, n, H, W, sides):
    fields = [oracle.mc_field(seed, f, H, W) for f in range(n)]
    return fields, np.array([oracle.mc_statistic(e, sides)[0] for e in fields])


def test_weights_balance_the_test():
    # with r2_s = (q sigma_s + mu_s)^4 a field meets every bound iff Q <= q, so
    # exactly ceil(alpha n) of the sample (ties aside) and about alpha of fresh
    # fields meet them all (Sec. 2.1)
    sides, H, W, n, alpha = [1, 2, 4, 8], 24, 24, 300, 0.9
    fields, Q = _sample(21, n, H, W, sides)
    q = oracle.order_quantile(Q, alpha)
    r2 = np.array([oracle.paper_bound(s * s, q) for s in sides])
    ok = sum(oracle.max_violation(e, sides, r2) <= 1e-12 for e in fields)
    k = math.ceil(alpha * n)
    assert k - 1 <= ok <= k
    fresh = [oracle.mc_field(22, f, H, W) for f in range(n)]
    ok2 = sum(oracle.max_violation(e, sides, r2) <= 0 for e in fresh) / n
    assert abs(ok2 - alpha) < 4.0 * math.sqrt(alpha * (1 - alpha) / n) + 1.0 / n


def test_single_window_quantile_is_chi_square_quantile():
    # one window of side s: the weight from the sampled q is the sampled
    # alpha-quantile of t ~ chi-square(s^2), within the DKW band
    s, n, alpha = 3, 3000, 0.9
    _, Q = _sample(8, n, s, s, [s])
    r2 = oracle.paper_bound(s * s, oracle.order_quantile(Q, alpha))
    eps = math.sqrt(math.log(2 / 1e-4) / (2 * n))
    assert abs(stats.chi2(s * s).cdf(r2) - alpha) < eps + 1.0 / n


# ---------------------------------------------------------------- planted mistakes

def _mutant(tmp_path, m):
    so = str(tmp_path / f"mc_mut{m}.so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
                           f"-DORACLE_MUTANT={m}", "-o", so,
                           os.path.join(os.path.dirname(oracle.__file__), "smre_oracle.c"),
                           "-lm"])
    L = ctypes.CDLL(so)
    base = oracle.lib()
    for name in ("oracle_philox4x64_10", "oracle_mc_field", "oracle_mc_statistic",
                 "oracle_order_quantile", "oracle_paper_bound"):
        getattr(L, name).argtypes = getattr(base, name).argtypes
        getattr(L, name).restype = getattr(base, name).restype
    return L


def test_pins_catch_planted_mistakes(tmp_path, monkeypatch):
    caught = {}
    for m in (5, 6, 7, 8, 9):
        monkeypatch.setattr(oracle, "_lib", _mutant(tmp_path, m))
        fails = 0
        for pin in (lambda: test_philox_matches_numpy([5, 17, 0, 0], [12345, 0]),
                    test_fields_are_standard_normal,
                    lambda: test_statistic_matches_brute_force(20, 17, [1, 4, 5, 16]),
                    lambda: test_single_window_statistic_inverts_paper_bound(3),
                    lambda: test_order_quantile_matches_numpy(101, 0.9)):
            try:
                pin()
            except AssertionError:
                fails += 1
        caught[m] = fails
    monkeypatch.setattr(oracle, "_lib", None)
    assert all(v > 0 for v in caught.values()), caught
