"""Pins for the full-Dykstra oracle (FP64, CPU).

The projection z = P(x0) onto {v : sum_S v^2 <= r2_S for every window S} has
no closed form in general (Sec. 2.2, P_G; Sec. 2.3, Algorithm 2), so the
oracle is pinned by what the mathematics fixes: closed forms where the family
degenerates, the KKT certificate, the variational inequality, a brute-force
QCQP solve on tiny images, symmetries, nonexpansiveness and order
independence.  A planted-mistake test rebuilds the oracle with one plausible
error at a time and checks that these pins catch it.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import qcqp
import smre_inputs as gi

TIGHT = 1e-14


def windows(H, W, sides):
    for s in sides:
        for i in range(H - s + 1):
            for j in range(W - s + 1):
                yield s, i, j


def bounds(sides, p=0.9):
    return oracle.chi2_bounds(sides, p)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("s", [1, 2, 3, 5])
def test_single_ball_is_a_rescale(s):
    """H = W = s, one side: the family is one ball, P is a rescale (Eq. dykstra:if)."""
    r2 = bounds([s])
    x0 = gi.gaussian(s, s, seed=s)
    x0 *= 2.0 * np.sqrt(r2[0] / np.sum(x0 * x0))
    z, sweeps, delta = oracle.dykstra(x0, [s], r2, tol=TIGHT, max_sweeps=10)
    n = float(np.sum(x0 * x0))
    expect = x0 * min(1.0, np.sqrt(r2[0] / n))
    assert n > r2[0]
    np.testing.assert_allclose(z, expect, rtol=5e-16, atol=0)  # n summed in another order
    assert sweeps == 2 and delta == 0.0


def test_side_one_is_a_clamp():
    """Side 1 only: the sets are disjoint pixels; one sweep clamps to +-sqrt(r2)."""
    x0 = gi.gaussian(9, 13, seed=3, scale=2.5)
    r2 = bounds([1])
    z, sweeps, delta = oracle.dykstra(x0, [1], r2, tol=TIGHT, max_sweeps=10)
    c = np.sqrt(r2[0])
    assert c == pytest.approx(1.6448536269514722, rel=1e-15)
    np.testing.assert_allclose(z, np.clip(x0, -c, c), rtol=1e-15, atol=0)
    assert sweeps == 2


def test_feasible_input_is_fixed():
    """A point inside every ball is its own projection; the increments stay zero."""
    sides = [1, 2, 3]
    r2 = bounds(sides)
    x0 = gi.gaussian(11, 7, seed=5)
    lim = min(np.sqrt(r2[k] / np.sum(x0[i:i + s, j:j + s] ** 2))
              for k, s in enumerate(sides) for _, i, j in windows(11, 7, [s]))
    x0 = x0 * min(1.0, 0.999 * lim)
    assert oracle.max_violation(x0, sides, r2) < 0
    z, sweeps, _, incs = oracle.dykstra(x0, sides, r2, tol=TIGHT, max_sweeps=5, want_incs=True)
    assert np.array_equal(z, x0)
    assert sweeps == 1
    assert not incs.any()


def test_idempotent():
    sides = [1, 2, 4]
    r2 = bounds(sides)
    x0 = gi.noise_blob(20, 20, seed=1)
    z, _, _ = oracle.dykstra(x0, sides, r2, tol=TIGHT, max_sweeps=20000)
    z2, sweeps, _ = oracle.dykstra(z, sides, r2, tol=TIGHT, max_sweeps=20000)
    np.testing.assert_allclose(z2, z, atol=1e-12)
    assert sweeps <= 3


# ---------------------------------------------------------------- certificates

@pytest.mark.parametrize("order,region", [(oracle.ORDER_DESC, 0), (oracle.ORDER_ASC, 0),
                                          (oracle.ORDER_REGION, 4)])
def test_kkt_certificate(order, region):
    """At the limit: x0 - z = sum_S I_S, I_S = mu_S z_S with mu_S >= 0, mu_S = 0
    on inactive windows, and z feasible.  With Slater (0 is interior) this
    certifies z = P(x0)."""
    sides = [1, 2, 3, 5]
    r2 = bounds(sides)
    x0 = gi.noise_blob(23, 19, seed=2)
    z, sweeps, delta, incs = oracle.dykstra(x0, sides, r2, tol=1e-13, max_sweeps=50000,
                                            order=order, region=region, want_incs=True)
    assert delta < 1e-13
    c = oracle.kkt(x0, z, incs, sides, r2, slack=1e-7)
    assert c["max_violation"] <= 1e-9
    assert c["sum_invariant"] <= 1e-12
    assert c["mult_residual"] <= 1e-9
    assert c["mu_min"] >= -1e-12
    assert c["inactive_inc"] <= 1e-9
    assert c["mu_max"] > 0  # some constraints are active


def test_invariant_after_every_sweep():
    """x + sum_S I_S = x0 holds after any number of sweeps (Dykstra's bookkeeping)."""
    sides = [2, 3, 4]
    r2 = bounds(sides)
    x0 = gi.noise_blob(17, 21, seed=4)
    for n in (1, 2, 7):
        z, _, _, incs = oracle.dykstra(x0, sides, r2, tol=0, max_sweeps=n, want_incs=True)
        c = oracle.kkt(x0, z, incs, sides, r2)
        assert c["sum_invariant"] <= 1e-13


def _feasible_scale(u, sides, r2):
    H, W = u.shape
    f = 1.0
    for k, s in enumerate(sides):
        for _, i, j in windows(H, W, [s]):
            n = np.sum(u[i:i + s, j:j + s] ** 2)
            if n > 0:
                f = min(f, np.sqrt(r2[k] / n))
    return u * f


def test_variational_inequality():
    """<x0 - z, y - z> <= 0 for every feasible y (projection onto a convex set)."""
    sides = [1, 2, 3]
    r2 = bounds(sides)
    x0 = gi.noise_blob(9, 10, seed=6, amp=6.0)
    z, _, _ = oracle.dykstra(x0, sides, r2, tol=1e-14, max_sweeps=100000)
    rng = np.random.default_rng(7)
    ys = [np.zeros_like(z), 0.5 * z, z * 0.99]
    for _ in range(200):
        ys.append(_feasible_scale(rng.standard_normal(z.shape) * rng.uniform(0.1, 5), sides, r2))
    for y in ys:
        assert np.sum((x0 - z) * (y - z)) <= 1e-9


# ---------------------------------------------------------------- brute force

def _qcqp(x0, sides, r2):
    return qcqp.project(x0, qcqp.all_windows(x0.shape[0], x0.shape[1], sides, r2))


@pytest.mark.parametrize("H,W,seed", [(4, 4, 0), (5, 5, 1), (4, 6, 2)])
def test_brute_force_qcqp(H, W, seed):
    sides = [1, 2, 3]
    r2 = bounds(sides)
    x0 = gi.gaussian(H, W, seed=seed, scale=3.0)
    z, _, _ = oracle.dykstra(x0, sides, r2, tol=1e-15, max_sweeps=200000)
    ref = _qcqp(x0, sides, r2)
    np.testing.assert_allclose(z, ref, atol=1e-10)


# ---------------------------------------------------------------- structure

def test_odd_symmetry_bitwise():
    sides = [1, 2, 4]
    r2 = bounds(sides)
    x0 = gi.noise_blob(16, 12, seed=8)
    a, _, _ = oracle.dykstra(x0, sides, r2, tol=0, max_sweeps=30)
    b, _, _ = oracle.dykstra(-x0, sides, r2, tol=0, max_sweeps=30)
    assert np.array_equal(a, -b)


def test_dihedral_symmetry():
    """The window family is invariant under flips and transposition, so P commutes
    with them (at the limit; the visiting order is not invariant)."""
    sides = [1, 2, 3]
    r2 = bounds(sides)
    x0 = gi.noise_blob(14, 14, seed=9)
    z, _, _ = oracle.dykstra(x0, sides, r2, tol=1e-14, max_sweeps=100000)
    for f in (np.flipud, np.fliplr, np.transpose):
        zf, _, _ = oracle.dykstra(np.ascontiguousarray(f(x0)), sides, r2, tol=1e-14,
                                  max_sweeps=100000)
        np.testing.assert_allclose(zf, f(z), atol=1e-11)


def test_nonexpansive():
    sides = [1, 2, 3]
    r2 = bounds(sides)
    a = gi.noise_blob(12, 12, seed=10)
    b = a + 0.3 * gi.gaussian(12, 12, seed=11)
    pa, _, _ = oracle.dykstra(a, sides, r2, tol=1e-14, max_sweeps=100000)
    pb, _, _ = oracle.dykstra(b, sides, r2, tol=1e-14, max_sweeps=100000)
    assert np.linalg.norm(pa - pb) <= np.linalg.norm(a - b) + 1e-12


def test_solid_set_shrinkage():
    """Each ball is sign-symmetric and downward closed in |v|, so |z_i| <= |x0_i|
    and z_i x0_i >= 0 at the projection."""
    sides = [1, 2, 4]
    r2 = bounds(sides)
    x0 = gi.emitters(32, 32, n_e=4, seed=12)
    z, _, _ = oracle.dykstra(x0, sides, r2, tol=1e-13, max_sweeps=100000)
    assert np.all(np.abs(z) <= np.abs(x0) + 1e-12)
    assert np.all(z * x0 >= -1e-24)


def test_order_independence():
    """Dykstra converges to the projection for any fixed cyclic order (Sec. 2.3)."""
    sides = [1, 2, 3, 4]
    r2 = bounds(sides)
    x0 = gi.noise_blob(21, 18, seed=13)
    ref, _, _ = oracle.dykstra(x0, sides, r2, tol=1e-14, max_sweeps=100000,
                               order=oracle.ORDER_DESC)
    for order, region in [(oracle.ORDER_ASC, 0), (oracle.ORDER_REGION, 3),
                          (oracle.ORDER_REGION, 5)]:
        z, _, _ = oracle.dykstra(x0, sides, r2, tol=1e-14, max_sweeps=100000, order=order,
                                 region=region)
        np.testing.assert_allclose(z, ref, atol=1e-10)


def test_region_order_equals_reordered_canonical_when_one_region():
    """With one region covering the image the region order is the canonical one."""
    sides = [1, 2, 3]
    r2 = bounds(sides)
    x0 = gi.noise_blob(9, 11, seed=14)
    a, _, _ = oracle.dykstra(x0, sides, r2, tol=0, max_sweeps=5, order=oracle.ORDER_DESC)
    b, _, _ = oracle.dykstra(x0, sides, r2, tol=0, max_sweeps=5, order=oracle.ORDER_REGION,
                             region=16)
    assert np.array_equal(a, b)


def test_rejects_bad_arguments():
    x0 = np.zeros((4, 4))
    with pytest.raises(ValueError):
        oracle.dykstra(x0, [5], [1.0])
    with pytest.raises(ValueError):
        oracle.dykstra(x0, [2, 2], [1.0, 1.0])
    with pytest.raises(ValueError):
        oracle.dykstra(x0, [2], [-1.0])
    with pytest.raises(ValueError):
        oracle.dykstra(x0, [1, 4], [1.0, 1.0], order=oracle.ORDER_REGION, region=2)


def test_window_count():
    assert oracle.window_count(64, 64, [1, 2, 4]) == 64 * 64 + 63 * 63 + 61 * 61
    assert oracle.window_count(1024, 1024, list(range(1, 17))) == 16532696


# ---------------------------------------------------------------- planted mistakes

def _mutant_lib(tmp_path, m):
    so = str(tmp_path / f"mut{m}.so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
                           f"-DORACLE_MUTANT={m}", "-o", so,
                           os.path.join(os.path.dirname(oracle.__file__), "smre_oracle.c"),
                           "-lm"])
    L = ctypes.CDLL(so)
    L.oracle_dykstra.argtypes = oracle.lib().oracle_dykstra.argtypes
    return L


@pytest.mark.parametrize("mutant", [1, 2, 3, 4])
def test_pins_catch_planted_mistakes(tmp_path, mutant):
    L = _mutant_lib(tmp_path, mutant)
    sides = np.array([1, 2, 3], dtype=np.int32)
    r2 = bounds(sides)
    x0 = gi.gaussian(4, 5, seed=0, scale=3.0)
    z = np.empty_like(x0)
    sw, dl = ctypes.c_int32(0), ctypes.c_double(0)
    rc = L.oracle_dykstra(oracle._d(x0), 4, 5, oracle._i(sides), 3, oracle._d(r2), 0, 0, 1e-15,
                          20000, oracle._d(z), None, ctypes.byref(sw), ctypes.byref(dl))
    assert rc == 0
    ref = _qcqp(x0, sides, r2)
    caught_bf = not np.allclose(z, ref, atol=1e-6)
    caught_feas = oracle.max_violation(z, sides, r2) > 1e-9
    assert caught_bf or caught_feas


# ---------------------------------------------------------------- threads

@pytest.mark.parametrize("order,region", [(oracle.ORDER_DESC, 0), (oracle.ORDER_ASC, 0),
                                          (oracle.ORDER_REGION, 8), (oracle.ORDER_REGION, 16)])
def test_threads_bitwise_equal(order, region):
    """The threaded sweeps split disjoint windows (one tiling) or disjoint region
    footprints (one colour): every thread count gives the same bits."""
    sides = [1, 2, 3, 5, 8]
    r2 = bounds(sides)
    x0 = gi.emitters(70, 83, n_e=12, seed=21)
    try:
        oracle.set_threads(1)
        a, sa, da, ia = oracle.dykstra(x0, sides, r2, tol=0, max_sweeps=6, order=order,
                                       region=region, want_incs=True)
        assert oracle.set_threads(4) == 4
        b, sb, db, ib = oracle.dykstra(x0, sides, r2, tol=0, max_sweeps=6, order=order,
                                       region=region, want_incs=True)
    finally:
        oracle.set_threads(1)
    assert np.array_equal(a, b) and np.array_equal(ia, ib) and da == db


# ---------------------------------------------------------------- warm start

def _converged(x0, sides, r2, **kw):
    return oracle.dykstra(x0, sides, r2, tol=1e-13, max_sweeps=50000, want_incs=True, **kw)


def test_warm_start_from_own_limit_stops_at_once():
    """Started from the converged increments of the same input, Dykstra starts at
    x0 - sum_S I_S = z (the invariant) and the first sweep changes nothing."""
    sides = [1, 2, 3, 5]
    r2 = bounds(sides)
    x0 = gi.noise_blob(23, 19, seed=2)
    z, _, d, incs = _converged(x0, sides, r2)
    assert d < 1e-13
    z2, sw, d2 = oracle.dykstra(x0, sides, r2, tol=1e-12, max_sweeps=100, incs0=incs)
    assert sw == 1 and d2 < 1e-12
    assert np.max(np.abs(z2 - z)) <= 1e-12


@pytest.mark.parametrize("order,region", [(oracle.ORDER_DESC, 0), (oracle.ORDER_REGION, 8)])
def test_warm_start_from_arbitrary_increments_reaches_projection(order, region):
    """Dykstra is block-coordinate minimisation of the dual of the projection, so
    any start reaches the same limit; the final state passes the KKT
    certificate and the invariant holds after every sweep."""
    sides = [1, 2, 3, 5]
    r2 = bounds(sides)
    x0 = gi.emitters(24, 29, n_e=4, seed=3)
    ref, _, _, _ = _converged(x0, sides, r2)
    rng = np.random.default_rng(7)
    T = oracle.ntilings(sides)
    inc0 = rng.normal(scale=0.5, size=(T,) + x0.shape)
    z1, _, _, i1 = oracle.dykstra(x0, sides, r2, tol=0, max_sweeps=3, order=order,
                                  region=region, incs0=inc0, want_incs=True)
    assert oracle.kkt(x0, z1, i1, sides, r2)["sum_invariant"] <= 1e-12
    z, sw, d, incs = oracle.dykstra(x0, sides, r2, tol=1e-13, max_sweeps=100000, order=order,
                                    region=region, incs0=inc0, want_incs=True)
    assert d < 1e-13
    assert np.max(np.abs(z - ref)) <= 1e-10
    c = oracle.kkt(x0, z, incs, sides, r2, slack=1e-7)
    assert c["max_violation"] <= 1e-9 and c["sum_invariant"] <= 1e-12
    assert c["mult_residual"] <= 1e-9 and c["mu_min"] >= -1e-12 and c["inactive_inc"] <= 1e-9


def test_warm_start_from_nearby_input_takes_fewer_sweeps():
    """Projecting a slightly moved input from the increments of the first
    projection (the situation of Algorithm 1's repeated projections) reaches
    the cold-start limit in fewer sweeps."""
    sides = [1, 2, 3, 4, 6]
    r2 = bounds(sides)
    x0 = gi.emitters(32, 36, n_e=6, seed=5)
    _, _, _, incs = oracle.dykstra(x0, sides, r2, tol=1e-10, max_sweeps=50000, want_incs=True)
    x1 = x0 + 0.01 * gi.gaussian(32, 36, seed=6)
    cold, sc, _ = oracle.dykstra(x1, sides, r2, tol=1e-10, max_sweeps=50000)
    warm, sw, _ = oracle.dykstra(x1, sides, r2, tol=1e-10, max_sweeps=50000, incs0=incs)
    assert sw < sc
    assert np.max(np.abs(warm - cold)) <= 1e-8


def test_warm_start_mutant_caught(tmp_path):
    """A warm start that keeps x = x0 (ignoring the given increments) converges
    to the projection of a different point; the same-limit pin catches it."""
    so = str(tmp_path / "mut10.so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
                           "-DORACLE_MUTANT=10", "-o", so,
                           os.path.join(os.path.dirname(oracle.__file__), "smre_oracle.c"),
                           "-lm"])
    L = ctypes.CDLL(so)
    L.oracle_dykstra_warm.argtypes = oracle.lib().oracle_dykstra_warm.argtypes
    sides = np.array([1, 2, 3], dtype=np.int32)
    r2 = bounds(sides)
    x0 = gi.emitters(12, 14, n_e=3, seed=8)
    ref, _, _ = oracle.dykstra(x0, sides, r2, tol=1e-13, max_sweeps=50000)
    inc = np.random.default_rng(1).normal(scale=0.5, size=(oracle.ntilings(sides), 12, 14))
    z = np.empty_like(x0)
    sw, dl = ctypes.c_int32(0), ctypes.c_double(0)
    rc = L.oracle_dykstra_warm(oracle._d(x0), 12, 14, oracle._i(sides), 3, oracle._d(r2), 0, 0,
                               1e-13, 50000, oracle._d(z), oracle._d(inc), ctypes.byref(sw),
                               ctypes.byref(dl))
    assert rc == 0
    assert np.max(np.abs(z - ref)) > 1e-6
