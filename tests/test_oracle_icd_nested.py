"""Pins for the nested-hierarchy ICD oracle (oracle_icd_nested): the ICD of
Sec. 3.2 with the square sides 2^k replaced by any divisor chain (e.g. 1, 3, 6,
12, 24, 48) and blocks up to 64 x 64 and beyond.

* The chain of powers of two is the paper's ICD: bitwise equal to
  oracle_icd_family (pinned in test_oracle_icd.py) for the same phases, up to
  K = 6.
* Composition of brute-force projections (generic NLP solver) on small images
  with non-power-of-two chains, a chain whose finest side is not 1, and shifts
  on each axis.
* At sizes the NLP solver cannot take (48- and 64-pixel blocks): every phase
  checked by an optimality certificate written from the KKT conditions of the
  projection onto nested balls (tests/nested_kkt.py), on the phase's input and
  output (prefix runs of the phase list).
* Closed forms: a one-level chain projects each block square onto its ball; a
  feasible input is fixed.  Symmetries: odd (bitwise), transpose (shifts
  swapped).  Planted mistakes in the oracle (a dropped level, the x shift taken
  from y, transposed increments) fail these pins.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import smre_inputs as gi
from nested_kkt import check_phase, phase_squares
from qcqp import project


def bounds(sides, p=0.9):
    return oracle.chi2_bounds(list(sides), p)


def squares_list(H, W, sides, r2, sy, sx, lo):
    sq = phase_squares(H, W, sides, sy, sx, lo)
    return [(y, x, sides[j], sides[j], r2[j]) for j in sq for (y, x) in sq[j]]


@pytest.mark.parametrize("K,phases", [(3, None), (6, None), (4, [(1, 0, 0), (0, 5, 1), (9, 2, 2)])])
def test_powers_of_two_chain_is_the_family(K, phases):
    sides = [1 << k for k in range(K + 1)]
    r2 = bounds(sides)
    ph = phases or oracle.icd_paper_phases(K)
    x0 = gi.emitters(70, 75, n_e=10, seed=K)
    a, na = oracle.icd_family(x0, K, r2, ph, tol=1e-11)
    b, nb = oracle.icd_nested(x0, sides, r2, ph, tol=1e-11)
    assert np.array_equal(a, b) and na == nb


@pytest.mark.parametrize("H,W,sides,phases", [
    (9, 10, [1, 3, 6], [(0, 0, 0), (3, 3, 0), (2, 4, 1)]),
    (8, 9, [2, 6], [(0, 0, 0), (3, 1, 0), (0, 4, 1)]),
    (7, 8, [1, 3], [(1, 2, 0), (0, 0, 1), (2, 0, 0)]),
    (10, 9, [1, 5], [(0, 0, 0), (2, 3, 0)]),
])
def test_phases_are_composed_projections(H, W, sides, phases):
    r2 = bounds(sides)
    x0 = gi.gaussian(H, W, seed=H * 11 + W, scale=2.5)
    z, _ = oracle.icd_nested(x0, sides, r2, phases, tol=1e-14)
    ref = x0.copy()
    for sy, sx, lo in phases:
        ref = project(ref, squares_list(H, W, sides, r2, sy, sx, lo))
    np.testing.assert_allclose(z, ref, atol=1e-9)


def _phase_io(x0, sides, r2, phases, tol=1e-14):
    """(input, output) of every phase, from prefix runs of the phase list."""
    outs = [x0]
    for p in range(1, len(phases) + 1):
        outs.append(oracle.icd_nested(x0, sides, r2, phases[:p], tol=tol)[0])
    return list(zip(outs[:-1], outs[1:]))


@pytest.mark.parametrize("H,W,sides,phases", [
    (60, 70, [1, 3, 6, 12, 24, 48], [(0, 0, 0), (3, 3, 0), (24, 0, 1), (6, 30, 3)]),
    (70, 75, [1, 2, 4, 8, 16, 32, 64], [(0, 0, 0), (2, 2, 1), (32, 32, 5), (1, 40, 0)]),
    (50, 53, [2, 6, 12], [(0, 0, 0), (6, 6, 0), (3, 9, 1)]),
])
def test_every_phase_meets_the_kkt_certificate(H, W, sides, phases):
    r2 = bounds(sides)
    # noise above the per-pixel bound makes the coarse squares bind too
    x0 = gi.emitters(H, W, n_e=max(4, H * W // 300), seed=H + W) + \
        1.3 * gi.gaussian(H, W, seed=H * W)
    act = np.zeros(len(sides), dtype=int)
    for (u, z), (sy, sx, lo) in zip(_phase_io(x0, sides, r2, phases), phases):
        for j, n in check_phase(u, z, sides, r2, sy, sx, lo).items():
            act[j] += n
    # the certificate was not vacuous: squares of the two coarsest levels bound
    assert act[-1] > 0 and act[-2] > 0, act


def test_certificate_rejects_a_wrong_phase():
    """The certificate itself: the right output of a different phase, or the
    right output nudged, fails it."""
    H, W, sides = 40, 44, [1, 3, 6, 12]
    r2 = bounds(sides)
    x0 = gi.gaussian(H, W, seed=4, scale=1.3)
    z0, _ = oracle.icd_nested(x0, sides, r2, [(0, 0, 0)], tol=1e-14)
    z1, _ = oracle.icd_nested(x0, sides, r2, [(6, 6, 0)], tol=1e-14)
    assert np.max(np.abs(z0 - z1)) > 0.1
    check_phase(x0, z0, sides, r2, 0, 0, 0)
    with pytest.raises(AssertionError):
        check_phase(x0, z1, sides, r2, 0, 0, 0)
    bad = z0.copy()
    i, j = np.unravel_index(np.argmax(np.abs(x0 - z0)), x0.shape)
    bad[i, j] *= 1.001
    with pytest.raises(AssertionError):
        check_phase(x0, bad, sides, r2, 0, 0, 0)


def test_one_level_is_a_ball_projection_per_square():
    H, W, L = 20, 23, 6
    r2 = bounds([L])
    x0 = gi.gaussian(H, W, seed=5, scale=3.0)
    for sy, sx in ((0, 0), (2, 5)):
        z, n = oracle.icd_nested(x0, [L], r2, [(sy, sx, 0)], tol=1e-14)
        ref = x0.copy()
        for (y, x) in phase_squares(H, W, [L], sy, sx, 0)[0]:
            blk = x0[y:y + L, x:x + L]
            nn = np.sum(blk * blk)
            if nn > r2[0]:
                ref[y:y + L, x:x + L] = blk * np.sqrt(r2[0] / nn)
        np.testing.assert_allclose(z, ref, rtol=1e-15, atol=0)


def test_feasible_input_is_fixed():
    x0 = gi.gaussian(30, 31, seed=2) * 0.2
    sides = [1, 3, 6, 12]
    z, _ = oracle.icd_nested(x0, sides, bounds(sides), [(0, 0, 0), (6, 6, 0)])
    assert np.array_equal(z, x0)


def test_odd_symmetry_bitwise_and_transpose():
    sides = [1, 3, 6, 12]
    r2 = bounds(sides)
    x0 = gi.emitters(30, 41, n_e=5, seed=8)
    ph = [(1, 0, 0), (0, 7, 1), (6, 2, 2)]
    a, _ = oracle.icd_nested(x0, sides, r2, ph, tol=1e-12)
    b, _ = oracle.icd_nested(-x0, sides, r2, ph, tol=1e-12)
    assert np.array_equal(a, -b)
    c, _ = oracle.icd_nested(np.ascontiguousarray(x0.T), sides, r2, [(x, y, l) for y, x, l in ph],
                             tol=1e-12)
    np.testing.assert_allclose(a, c.T, rtol=0, atol=1e-11)


@pytest.mark.parametrize("sides,phases", [
    ([2, 3], [(0, 0, 0)]),      # 2 does not divide 3
    ([3, 3], [(0, 0, 0)]),      # not ascending
    ([1, 3], [(3, 0, 0)]),      # shift >= block side
    ([1, 3], [(0, 0, 2)]),      # no level 2
    ([0, 3], [(0, 0, 0)]),
])
def test_rejects_bad_arguments(sides, phases):
    with pytest.raises(ValueError):
        oracle.icd_nested(np.zeros((8, 8)), sides, [1.0] * len(sides), phases)


def _mutant(tmp_path, m):
    so = str(tmp_path / f"mut{m}.so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
                           f"-DORACLE_MUTANT={m}", "-o", so,
                           os.path.join(os.path.dirname(oracle.__file__), "smre_oracle.c"),
                           "-lm"])
    L = ctypes.CDLL(so)
    for name in ("oracle_icd_nested", "oracle_chi2_quantile", "oracle_chi2_cdf"):
        getattr(L, name).argtypes = getattr(oracle.lib(), name).argtypes
        getattr(L, name).restype = getattr(oracle.lib(), name).restype
    return L


@pytest.mark.parametrize("mutant", [11, 12, 13])
def test_pins_catch_planted_mistakes(tmp_path, monkeypatch, mutant):
    monkeypatch.setattr(oracle, "_lib", _mutant(tmp_path, mutant))
    caught = 0
    for case in ((9, 10, [1, 3, 6], [(0, 0, 0), (3, 3, 0), (2, 4, 1)]),
                 (8, 9, [2, 6], [(0, 0, 0), (3, 1, 0), (0, 4, 1)])):
        try:
            test_phases_are_composed_projections(*case)
        except AssertionError:
            caught += 1
    try:
        test_every_phase_meets_the_kkt_certificate(
            60, 70, [1, 3, 6, 12, 24, 48], [(0, 0, 0), (3, 3, 0), (24, 0, 1), (6, 30, 3)])
    except AssertionError:
        caught += 1
    assert caught >= 2
