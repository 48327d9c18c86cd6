"""Optimality certificate for a projection onto nested square balls, written
from the KKT conditions alone (independent of Dykstra and of the oracle).

Phase p of a nested ICD projects its input u onto C = {z : sum_S z^2 <= r2_S}
over the squares S of the phase.  z = P_C(u) iff z is feasible and there are
multipliers m_S >= 0, zero on inactive squares, with u_i = z_i (1 + sum_{S
containing i} m_S) at every pixel.  So rho_i = u_i / z_i - 1 must be a sum of
nonnegative multipliers along the chain of squares containing pixel i.  The
squares form a forest (each lies in one square of the next level, when that
square is inside the image), and existence of such multipliers is decided
bottom-up: the set of admissible "sum of the ancestors' multipliers" values of
a subtree is an interval -- at a pixel [rho_i - eps_i, rho_i + eps_i]; at a
square, the intersection I of its children's sets if inactive, or (-inf,
max I] if active (its own multiplier absorbs any shortfall) -- and every root
must admit 0.
"""
import numpy as np


def phase_squares(H, W, sides, sy, sx, lo):
    """{level: [(y, x)]} of the squares of one phase inside the image."""
    B = sides[-1]
    oy = sy - B if sy else 0
    ox = sx - B if sx else 0
    out = {}
    for j in range(lo, len(sides)):
        L = sides[j]
        out[j] = [(y, x) for y in range(oy, H, L) for x in range(ox, W, L)
                  if y >= 0 and x >= 0 and y + L <= H and x + L <= W]
    return out


def check_phase(u, z, sides, r2, sy, sx, lo, delta_rel=1e-10, act_rel=1e-8, feas_rel=1e-9):
    """Raises AssertionError unless z is P_C(u) for the phase (sy, sx, lo) to
    the given tolerances; returns {level: number of active squares}."""
    H, W = u.shape
    umax = float(np.max(np.abs(u))) or 1.0
    delta = delta_rel * umax
    nz = z != 0
    assert np.all(nz | (np.abs(u) <= delta)), "a pixel was zeroed that was not zero"
    with np.errstate(divide="ignore", invalid="ignore"):
        rho = np.where(nz, u / np.where(nz, z, 1.0) - 1.0, 0.0)
        eps = np.where(nz, (1.0 + np.abs(rho)) * delta / np.abs(np.where(nz, z, 1.0)), np.inf)
    plo, phi = rho - eps, rho + eps
    sq = phase_squares(H, W, sides, sy, sx, lo)
    F = {}
    covered = np.zeros((H, W), dtype=bool)
    consumed = set()
    active = {j: 0 for j in range(lo, len(sides))}
    for j in range(lo, len(sides)):
        L = sides[j]
        for (y, x) in sq[j]:
            n2 = float(np.sum(z[y:y + L, x:x + L] ** 2))
            assert n2 <= r2[j] * (1 + feas_rel), ("infeasible", j, y, x, n2 / r2[j] - 1)
            if j == lo:
                a = float(np.max(plo[y:y + L, x:x + L]))
                b = float(np.min(phi[y:y + L, x:x + L]))
                covered[y:y + L, x:x + L] = True
            else:
                Lc = sides[j - 1]
                a, b = -np.inf, np.inf
                for yy in range(y, y + L, Lc):
                    for xx in range(x, x + L, Lc):
                        ca, cb = F[(j - 1, yy, xx)]
                        a, b = max(a, ca), min(cb, b)
                        consumed.add((j - 1, yy, xx))
            assert a <= b, ("no multipliers", j, y, x, a, b)
            if n2 >= r2[j] * (1 - act_rel):
                F[(j, y, x)] = (-np.inf, b)
                active[j] += 1
            else:
                F[(j, y, x)] = (a, b)
    for key, (a, b) in F.items():
        if key not in consumed:
            assert a <= 0 <= b, ("root", key, a, b)
    bare = ~covered
    assert np.all(plo[bare] <= 0) and np.all(phi[bare] >= 0), "a pixel outside every square moved"
    return active
