"""Brute-force projection onto an intersection of window balls by a generic
NLP solver (SciPy SLSQP).  Independent of Dykstra: used to pin the oracle."""
import numpy as np
from scipy.optimize import minimize


def project(x0, squares, ftol=1e-12):
    """argmin 0.5||v - x0||^2 s.t. sum_{S} v^2 <= r2 for each (i, j, h, w, r2)."""
    H, W = x0.shape

    def cons_f(v):
        v = v.reshape(H, W)
        return np.array([r2 - np.sum(v[i:i + h, j:j + w] ** 2) for i, j, h, w, r2 in squares])

    def cons_j(v):
        v = v.reshape(H, W)
        J = np.zeros((len(squares), H * W))
        for r, (i, j, h, w, _) in enumerate(squares):
            g = np.zeros((H, W))
            g[i:i + h, j:j + w] = -2 * v[i:i + h, j:j + w]
            J[r] = g.ravel()
        return J

    # Start strictly inside the feasible set, off the origin (where every
    # constraint gradient vanishes and the linearised problem degenerates).
    f = 1.0
    for i, j, h, w, r2 in squares:
        n = np.sum(x0[i:i + h, j:j + w] ** 2)
        if n > 0:
            f = min(f, np.sqrt(r2 / n))
    start = (0.5 * f * x0).ravel()
    best = None
    for tol in (ftol, 10 * ftol, 100 * ftol, 0.1 * ftol):
        res = minimize(lambda v: 0.5 * np.sum((v - x0.ravel()) ** 2), start,
                       jac=lambda v: v - x0.ravel(), method="SLSQP",
                       constraints=[{"type": "ineq", "fun": cons_f, "jac": cons_j}],
                       options={"ftol": tol, "maxiter": 3000})
        if best is None or np.min(cons_f(res.x)) > np.min(cons_f(best.x)) - 1e-6:
            best = res
        if res.success:
            break
    return _polish(x0, squares, best.x.reshape(H, W))


def _polish(x0, squares, v, active_tol=1e-6, iters=30):
    """Newton on the KKT system of the constraints active at v:
    v - x0 + 2 sum_A lam_S (v on S) = 0,  sum_S v^2 = r2_S (S in A).
    SLSQP's line search stalls near 1e-8; this brings the point to rounding
    level when the active set is identified correctly, and checks lam >= 0."""
    H, W = x0.shape
    n = H * W
    masks, r2s = [], []
    for i, j, h, w, r2 in squares:
        if abs(np.sum(v[i:i + h, j:j + w] ** 2) - r2) <= active_tol * r2:
            m = np.zeros((H, W), dtype=bool)
            m[i:i + h, j:j + w] = True
            masks.append(m.ravel())
            r2s.append(r2)
    if not masks:
        return x0.copy() if all(np.sum(x0[i:i + h, j:j + w] ** 2) <= r2
                                for i, j, h, w, r2 in squares) else v
    M = np.array(masks, dtype=float)  # m x n
    r2s = np.array(r2s)
    x = v.ravel().copy()
    g = x0.ravel()
    lam = np.linalg.lstsq((2 * M * x).T, g - x, rcond=None)[0]
    for _ in range(iters):
        F1 = x - g + 2 * (M.T @ lam) * x
        F2 = M @ (x * x) - r2s
        if max(np.max(np.abs(F1)), np.max(np.abs(F2))) < 1e-15:
            break
        J = np.zeros((n + len(r2s), n + len(r2s)))
        J[:n, :n] = np.diag(1 + 2 * (M.T @ lam))
        J[:n, n:] = (2 * M * x).T
        J[n:, :n] = 2 * M * x
        d = np.linalg.lstsq(J, -np.concatenate([F1, F2]), rcond=None)[0]
        x += d[:n]
        lam += d[n:]
    assert np.min(lam) > -1e-9, "negative multiplier: wrong active set"
    out = x.reshape(H, W)
    for i, j, h, w, r2 in squares:
        assert np.sum(out[i:i + h, j:j + w] ** 2) <= r2 * (1 + 1e-12)
    return out


def all_windows(H, W, sides, r2):
    return [(i, j, s, s, r) for s, r in zip(sides, r2)
            for i in range(H - s + 1) for j in range(W - s + 1)]
