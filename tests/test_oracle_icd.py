"""Pins for the incomplete-Dykstra (ICD) oracle, Sec. 3.2.

ICD is defined by its algorithm: phase i projects onto C_i, the intersection
of the balls of the squares of side 2^k (k = i..K) on the lattice shifted by
2^i mod 2^K, and the phases are composed in order.  The pins: the composition
of brute-force projections, closed forms (K = 0 clamps; feasible input is
fixed), feasibility for every ICD set, symmetry, and the comparison with the
projection onto the whole ICD family.
"""
import numpy as np
import pytest

import oracle
import smre_inputs as gi
from qcqp import project


def icd_bounds(K, p=0.9):
    return oracle.chi2_bounds([1 << k for k in range(K + 1)], p)


def phase_squares(H, W, K, i, r2):
    """Squares of phase i: side 2^k (k = i..K) on the lattice offset o = 2^i mod 2^K,
    inside the image."""
    B = 1 << K
    o = (1 << i) % B
    out = []
    for k in range(i, K + 1):
        L = 1 << k
        start = o - B if o else 0
        for y in range(start, H, L):
            for x in range(start, W, L):
                if y >= 0 and x >= 0 and y + L <= H and x + L <= W:
                    out.append((y, x, L, L, r2[k]))
    return out


def test_k0_is_a_clamp():
    r2 = icd_bounds(0)
    x0 = gi.gaussian(7, 9, seed=1, scale=2.0)
    z, _ = oracle.icd(x0, 0, r2)
    c = np.sqrt(r2[0])
    np.testing.assert_allclose(z, np.clip(x0, -c, c), rtol=3e-16, atol=0)


def test_feasible_input_is_fixed():
    K = 3
    r2 = icd_bounds(K)
    x0 = gi.gaussian(16, 16, seed=2) * 0.2
    z, inner = oracle.icd(x0, K, r2)
    assert np.array_equal(z, x0)


@pytest.mark.parametrize("H,W,K", [(8, 8, 2), (7, 9, 2), (6, 6, 1)])
def test_phases_are_composed_projections(H, W, K):
    """ICD = P_{C_K} o ... o P_{C_0}; each P_{C_i} checked by a generic solver."""
    r2 = icd_bounds(K)
    x0 = gi.gaussian(H, W, seed=H * 10 + W, scale=2.5)
    z, _ = oracle.icd(x0, K, r2, tol=1e-14)
    ref = x0.copy()
    for i in range(K + 1):
        ref = project(ref, phase_squares(H, W, K, i, r2))
    np.testing.assert_allclose(z, ref, atol=1e-10)


def test_first_phase_alone():
    H, W, K = 8, 8, 2
    r2 = icd_bounds(K)
    x0 = gi.gaussian(H, W, seed=5, scale=3.0)
    z, _ = oracle.icd(x0, K, r2, tol=1e-14, num_phases=1)
    np.testing.assert_allclose(z, project(x0, phase_squares(H, W, K, 0, r2)), atol=1e-10)


@pytest.mark.parametrize("H,W,K", [(64, 64, 3), (37, 45, 3), (64, 48, 4)])
def test_output_feasible_for_every_icd_set(H, W, K):
    """Later phases never increase |x_i| (each ball is a solid set), so the
    output satisfies every constraint of every phase, not only the last."""
    r2 = icd_bounds(K)
    x0 = gi.emitters(H, W, n_e=max(2, H * W // 500), seed=7)
    z, _ = oracle.icd(x0, K, r2, tol=1e-14)
    worst = -1.0
    for i in range(K + 1):
        for (y, x, h, w, r) in phase_squares(H, W, K, i, r2):
            worst = max(worst, np.sum(z[y:y + h, x:x + w] ** 2) / r - 1)
    assert worst <= 1e-9
    assert np.all(np.abs(z) <= np.abs(x0) + 1e-12)


def test_transpose_symmetry():
    K = 3
    r2 = icd_bounds(K)
    x0 = gi.emitters(40, 40, n_e=6, seed=8)
    z, _ = oracle.icd(x0, K, r2, tol=1e-14)
    zt, _ = oracle.icd(np.ascontiguousarray(x0.T), K, r2, tol=1e-14)
    np.testing.assert_allclose(zt, z.T, atol=1e-12)


def test_odd_symmetry_bitwise():
    K = 3
    r2 = icd_bounds(K)
    x0 = gi.emitters(24, 40, n_e=6, seed=9)
    a, _ = oracle.icd(x0, K, r2, tol=1e-6)
    b, _ = oracle.icd(-x0, K, r2, tol=1e-6)
    assert np.array_equal(a, -b)


def test_not_closer_than_projection_onto_family():
    """ICD lands in the ICD family's feasible set, so it is no closer to x0 than
    the projection onto that set."""
    H, W, K = 8, 8, 2
    r2 = icd_bounds(K)
    x0 = gi.gaussian(H, W, seed=11, scale=3.0)
    z, _ = oracle.icd(x0, K, r2, tol=1e-14)
    fam = sum((phase_squares(H, W, K, i, r2) for i in range(K + 1)), [])
    p = project(x0, fam)
    assert np.linalg.norm(x0 - z) >= np.linalg.norm(x0 - p) - 1e-7


def test_paper_tolerance_mode_close_to_tight():
    K = 3
    r2 = icd_bounds(K)
    x0 = gi.emitters(64, 64, n_e=8, seed=12)
    tight, _ = oracle.icd(x0, K, r2, tol=1e-14)
    loose, n = oracle.icd(x0, K, r2, tol=1e-3, mode=oracle.TOL_MEANABS)
    assert np.max(np.abs(loose - tight)) < 0.05
    assert n >= 4  # at least one inner sweep per block and phase


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.icd(np.zeros((8, 8)), 2, [1.0, 1.0])
    with pytest.raises(ValueError):
        oracle.icd(np.zeros((8, 8)), 2, [1.0, 1.0, -1.0])
    with pytest.raises(ValueError):
        oracle.icd(np.zeros((8, 8)), 2, [1.0, 1.0, 1.0], num_phases=4)


# ---------------------------------------------------------------- phase families

def family_squares(H, W, K, sy, sx, lo, r2):
    """Squares of one phase of a family: side 2^k (k = lo..K) on the lattice
    shifted by (sy, sx), inside the image."""
    B = 1 << K
    out = []
    for k in range(lo, K + 1):
        L = 1 << k
        y0 = sy - B if sy else 0
        x0 = sx - B if sx else 0
        for y in range(y0, H, L):
            for x in range(x0, W, L):
                if y >= 0 and x >= 0 and y + L <= H and x + L <= W:
                    out.append((y, x, L, L, r2[k]))
    return out


def test_paper_family_is_the_icd():
    K = 3
    r2 = icd_bounds(K)
    x0 = gi.emitters(40, 36, n_e=6, seed=3)
    a, na = oracle.icd(x0, K, r2, tol=1e-12)
    b, nb = oracle.icd_family(x0, K, r2, oracle.icd_paper_phases(K), tol=1e-12)
    assert np.array_equal(a, b) and na == nb


@pytest.mark.parametrize("H,W,K,phases", [
    (8, 8, 2, [(1, 0, 0), (0, 1, 0), (2, 2, 1)]),
    (7, 9, 2, [(0, 0, 0), (1, 0, 1), (0, 3, 1)]),
    (6, 7, 1, [(1, 0, 0), (0, 1, 1)]),
])
def test_family_phases_are_composed_projections(H, W, K, phases):
    """Off-diagonal families: the composition of brute-force projections onto
    each phase's set (a mix-up of the two axes fails here)."""
    r2 = icd_bounds(K)
    x0 = gi.gaussian(H, W, seed=H * 7 + W, scale=2.5)
    z, _ = oracle.icd_family(x0, K, r2, phases, tol=1e-14)
    ref = x0.copy()
    for sy, sx, lo in phases:
        ref = project(ref, family_squares(H, W, K, sy, sx, lo, r2))
    np.testing.assert_allclose(z, ref, atol=1e-10)


def test_family_transpose_swaps_shifts():
    K = 3
    r2 = icd_bounds(K)
    x0 = gi.emitters(30, 41, n_e=5, seed=8)
    ph = [(1, 0, 0), (0, 2, 1), (4, 1, 2)]
    a, _ = oracle.icd_family(x0, K, r2, ph, tol=1e-13)
    b, _ = oracle.icd_family(np.ascontiguousarray(x0.T), K, r2, [(x, y, l) for y, x, l in ph],
                             tol=1e-13)
    np.testing.assert_allclose(a, b.T, rtol=0, atol=1e-12)


def test_family_rejects_bad_phases():
    with pytest.raises(ValueError):
        oracle.icd_family(np.zeros((8, 8)), 2, [1.0] * 3, [(4, 0, 0)])
    with pytest.raises(ValueError):
        oracle.icd_family(np.zeros((8, 8)), 2, [1.0] * 3, [(0, 0, 3)])
