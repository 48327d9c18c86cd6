"""Pins of the oracle's ADMM outer loop (Sec. 2.2, Algorithm 1, split form).

* The PSF operator is symmetric (the x-step uses A^T = A).
* A = identity: the problem min lam/2 ||x||^2 s.t. I - x in tau_G has the
  closed-form solution x = I - P_G(I), eps = P_G(I); the iteration reaches it.
* Blurring A: at the fixed point the multipliers certify optimality (KKT):
  I = A x + eps, eps in tau_G, eps = P_G(eps + Y1/rho1) (Y1/rho1 is normal to
  the feasible set at eps), lam x = A^T Y1, z = x.
* Inactive constraint (P_G = identity): x -> 0, eps -> I.
"""
import numpy as np
import pytest

import oracle
import oracle.admm as ad
import smre_inputs as gi


def test_blur_is_symmetric():
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal((2, 23, 31))
    for sigma in (0.7, 2.0, 4.0):
        lhs = np.vdot(ad.blur(u, sigma), v)
        rhs = np.vdot(u, ad.blur(v, sigma))
        assert lhs == pytest.approx(rhs, rel=1e-12)


def test_identity_operator_reaches_closed_form():
    I = gi.gaussian(12, 12, seed=3, scale=1.5)
    sides = [1, 2, 4]
    r2 = oracle.chi2_bounds(sides)
    P = lambda X: ad.project_full(X, sides, r2, 1e-12)  # noqa: E731
    out = ad.admm(I, 0.0, P, delta=1e-10, max_iter=400)
    eps_star = P(I)
    np.testing.assert_allclose(out["x"], I - eps_star, atol=1e-7)
    np.testing.assert_allclose(out["eps"], eps_star, atol=1e-7)
    np.testing.assert_allclose(out["z"], out["x"], atol=1e-6)


def test_blur_fixed_point_satisfies_kkt():
    # dual steps equal to the penalties (alpha = rho) so the iteration reaches
    # its fixed point within a couple of thousand steps
    H, W, sigma, lam, rho1, rho2 = 8, 9, 0.8, 1.0, 6.192, 1.8
    I = gi.gaussian(H, W, seed=5, scale=2.0)
    sides = [1, 2]
    r2 = oracle.chi2_bounds(sides)
    P = lambda X: ad.project_full(X, sides, r2, 1e-13)  # noqa: E731
    out = ad.admm(I, sigma, P, lam=lam, rho1=rho1, rho2=rho2, alpha1=rho1, alpha2=rho2,
                  delta=1e-11, max_iter=3000)
    assert out["iterations"] < 3000
    x, eps, Y1 = out["x"], out["eps"], out["Y1"]
    assert np.abs(I - ad.blur(x, sigma) - eps).max() < 1e-10
    assert oracle.max_violation(eps, sides, r2) <= 1e-9
    np.testing.assert_allclose(P(eps + Y1 / rho1), eps, atol=1e-10)
    np.testing.assert_allclose(lam * x, ad.blur(Y1, sigma), atol=1e-10)
    np.testing.assert_allclose(out["z"], x, atol=1e-10)


def test_inactive_constraint_drives_x_to_zero():
    I = gi.gaussian(10, 11, seed=2)
    out = ad.admm(I, 1.5, lambda X: X, delta=1e-12, max_iter=3000)
    assert np.abs(out["x"]).max() < 1e-8
    np.testing.assert_allclose(out["eps"], I, atol=1e-8)
