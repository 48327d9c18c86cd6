"""ADMM outer loop of the SMRE (TEST INFRASTRUCTURE, FP64, plain numpy).

Sec. 2.2 of the paper: minimise G(eps) + R(z) subject to I = A*x + eps and
z = x (the split form, Eq. (eq3)) with the augmented Lagrangian of Eq. (eq2)
extended by the second constraint (multipliers Y1, Y2, penalties rho1, rho2).
One iteration (Algorithm 1, in the order x, eps, z, multipliers):

  x-step   the linearised update with stabilisation gamma: the quadratic
           coupling terms are linearised at the current x and a proximal term
           gamma ||x - x_r||^2 is added, so
             grad = -A^T (rho1 (I - A x_r - eps) + Y1) + rho2 (x_r - z) + Y2,
             x_{r+1} = x_r - grad / (2 gamma);
  eps-step eps = P_G(I - A x_{r+1} + Y1 / rho1), the projection onto the
           multi-resolution constraint (Sec. 2.2, last equation), by full
           Dykstra or by the incomplete variant (Sec. 3.2);
  z-step   argmin_z R(z) + rho2/2 ||z - (x + Y2/rho2)||^2 with the generic L2
           regulariser R(z) = lam/2 ||z||^2 (Sec. 4 uses it for the SOFI data):
             z = (rho2 x + Y2) / (lam + rho2);
  Y-steps  steepest ascent: Y1 += alpha1 (I - A x - eps), Y2 += alpha2 (x - z).

Stop once ||x_{r+1} - x_r||_2 <= delta and ||I - A x - eps||_2 <= delta, or
after max_iter iterations.  A is the Gaussian PSF: scipy's gaussian_filter
with zero boundary (mode 'constant', truncate 4), a symmetric operator, so
A^T = A.
"""
import numpy as np
from scipy.ndimage import gaussian_filter

from . import dykstra as _dykstra
from . import icd as _icd
from . import ORDER_DESC, TOL_MEANABS


def blur(u, sigma):
    """A u: Gaussian PSF of width sigma px, zero outside the image."""
    if sigma <= 0:
        return u.copy()
    return gaussian_filter(u, sigma, mode="constant", truncate=4.0)


def project_full(X, sides, r2, tol):
    z, _, _ = _dykstra(X, sides, r2, tol=tol, max_sweeps=100000, order=ORDER_DESC)
    return z


def project_icd(X, K, r2, tol, mode=TOL_MEANABS):
    z, _ = _icd(X, K, r2, tol=tol, mode=mode, max_inner=100000)
    return z


def admm(I, sigma, project, lam=1.0, rho1=6.192, rho2=1.8, alpha1=1.2, alpha2=0.12,
         gamma=None, delta=1e-3, max_iter=100, x0=None):
    """Returns a dict: x, eps, z, Y1, Y2, iterations and history, where
    history[r] = (||x_{r+1} - x_r||_2, ||I - A x - eps||_2).  x starts at 0
    (eps, z, Y1, Y2 too).  project(X) -> P_G(X)."""
    I = np.asarray(I, dtype=np.float64)
    if gamma is None:
        gamma = 0.5 * (rho1 + rho2)
    x = np.zeros_like(I) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    eps = np.zeros_like(I)
    z = x.copy()
    Y1 = np.zeros_like(I)
    Y2 = np.zeros_like(I)
    hist = []
    it = 0
    for it in range(1, max_iter + 1):
        Ax = blur(x, sigma)
        grad = -blur(rho1 * (I - Ax - eps) + Y1, sigma) + rho2 * (x - z) + Y2
        x_new = x - grad / (2.0 * gamma)
        dx = float(np.linalg.norm(x_new - x))
        x = x_new
        Ax = blur(x, sigma)
        eps = project(I - Ax + Y1 / rho1)
        z = (rho2 * x + Y2) / (lam + rho2)
        res = I - Ax - eps
        Y1 = Y1 + alpha1 * res
        Y2 = Y2 + alpha2 * (x - z)
        rn = float(np.linalg.norm(res))
        hist.append((dx, rn))
        if dx <= delta and rn <= delta:
            break
    return {"x": x, "eps": eps, "z": z, "Y1": Y1, "Y2": Y2, "iterations": it, "history": hist}
