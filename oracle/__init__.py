"""Python view of the FP64 CPU oracle (TEST INFRASTRUCTURE).

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this package.  The HIP library shares no code with it.  See smre_oracle.c for
the paper passages each routine follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

ORDER_DESC = 0
ORDER_ASC = 1
ORDER_REGION = 2
TOL_MAXABS = 0
TOL_MEANABS = 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        i64 = ctypes.c_int64
        L.oracle_chi2_cdf.argtypes = [ctypes.c_int, ctypes.c_double]
        L.oracle_chi2_cdf.restype = ctypes.c_double
        L.oracle_chi2_quantile.argtypes = [ctypes.c_int, ctypes.c_double]
        L.oracle_chi2_quantile.restype = ctypes.c_double
        L.oracle_paper_bound.argtypes = [i64, ctypes.c_double]
        L.oracle_paper_bound.restype = ctypes.c_double
        L.oracle_dykstra.argtypes = [dp, i64, i64, ip, ctypes.c_int32, dp, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_double, ctypes.c_int32, dp, dp,
                                     ip, dp]
        L.oracle_dykstra.restype = ctypes.c_int
        L.oracle_dykstra_warm.argtypes = L.oracle_dykstra.argtypes
        L.oracle_dykstra_warm.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = ctypes.c_int
        L.oracle_window_count.argtypes = [i64, i64, ip, ctypes.c_int32]
        L.oracle_window_count.restype = i64
        L.oracle_max_violation.argtypes = [dp, i64, i64, ip, ctypes.c_int32, dp]
        L.oracle_max_violation.restype = ctypes.c_double
        L.oracle_kkt.argtypes = [dp, dp, dp, i64, i64, ip, ctypes.c_int32, dp, ctypes.c_double,
                                 dp]
        L.oracle_kkt.restype = ctypes.c_int
        L.oracle_icd.argtypes = [dp, i64, i64, ctypes.c_int32, dp, ctypes.c_double,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp,
                                 ctypes.POINTER(ctypes.c_int64)]
        L.oracle_icd.restype = ctypes.c_int
        L.oracle_icd_family.argtypes = [dp, i64, i64, ctypes.c_int32, dp, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ip, ip,
                                        ip, dp, ctypes.POINTER(ctypes.c_int64)]
        L.oracle_icd_family.restype = ctypes.c_int
        L.oracle_icd_nested.argtypes = [dp, i64, i64, ctypes.c_int32, ip, dp, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ip, ip,
                                        ip, dp, ctypes.POINTER(ctypes.c_int64)]
        L.oracle_icd_nested.restype = ctypes.c_int
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.oracle_philox4x64_10.restype = None
        L.oracle_mc_field.argtypes = [ctypes.c_uint64, i64, i64, i64, dp]
        L.oracle_mc_field.restype = None
        L.oracle_mc_statistic.argtypes = [dp, i64, i64, ip, ctypes.c_int32, dp]
        L.oracle_mc_statistic.restype = ctypes.c_double
        L.oracle_order_quantile.argtypes = [dp, i64, ctypes.c_double]
        L.oracle_order_quantile.restype = ctypes.c_double
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def chi2_cdf(k, x):
    return lib().oracle_chi2_cdf(int(k), float(x))


def chi2_quantile(k, p):
    return lib().oracle_chi2_quantile(int(k), float(p))


def chi2_bounds(sides, p=0.9):
    """r2_s = chi-square(s*s dof) p-quantile for each side s."""
    return np.array([chi2_quantile(s * s, p) for s in sides], dtype=np.float64)


def paper_bound(npix, q_alpha):
    return lib().oracle_paper_bound(int(npix), float(q_alpha))


def ntilings(sides):
    return int(sum(int(s) * int(s) for s in sides))


def set_threads(n):
    """Worker threads of the sweeps (1 = sequential).  Every count gives
    bitwise the same iterates (the threads take disjoint windows / regions).
    Returns the count in effect."""
    return lib().oracle_set_threads(int(n))


def dykstra(x0, sides, r2, tol=1e-10, max_sweeps=500, order=ORDER_DESC, region=0,
            want_incs=False, incs0=None, in_place=False):
    """Full Dykstra in FP64.  Returns (z, sweeps, last_delta[, incs]).

    tol <= 0 runs exactly max_sweeps sweeps.  incs has shape (T, H, W) with
    tilings indexed sides-descending, then offset row a, then offset column b.
    incs0 (same shape) starts Dykstra from those increments instead of zero
    (x starts at x0 - sum_S I_S); it is not modified unless in_place is set
    (then it must be a C-contiguous float64 array and receives the final
    increments, which saves a copy of a large state).
    """
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    H, W = x0.shape
    sides = np.ascontiguousarray(sides, dtype=np.int32)
    r2 = np.ascontiguousarray(r2, dtype=np.float64)
    z = np.empty_like(x0)
    incs = None
    if incs0 is not None and in_place:
        if incs0.dtype != np.float64 or not incs0.flags.c_contiguous:
            raise ValueError("in_place needs a C-contiguous float64 incs0")
        incs = incs0
    elif incs0 is not None:
        incs = np.array(incs0, dtype=np.float64, order="C", copy=True)
    if incs0 is not None:
        if incs.shape != (ntilings(sides), H, W):
            raise ValueError("incs0 must have shape (T, H, W)")
    elif want_incs:
        incs = np.empty((ntilings(sides), H, W), dtype=np.float64)
    sw = ctypes.c_int32(0)
    dl = ctypes.c_double(0)
    fn = lib().oracle_dykstra_warm if incs0 is not None else lib().oracle_dykstra
    rc = fn(_d(x0), H, W, _i(sides), len(sides), _d(r2), int(order), int(region), float(tol),
            int(max_sweeps), _d(z), _d(incs) if incs is not None else None, ctypes.byref(sw),
            ctypes.byref(dl))
    if rc != 0:
        raise ValueError("oracle_dykstra rejected its arguments")
    if want_incs:
        return z, sw.value, dl.value, incs
    return z, sw.value, dl.value


def window_count(H, W, sides):
    sides = np.ascontiguousarray(sides, dtype=np.int32)
    return lib().oracle_window_count(H, W, _i(sides), len(sides))


def max_violation(z, sides, r2):
    z = np.ascontiguousarray(z, dtype=np.float64)
    sides = np.ascontiguousarray(sides, dtype=np.int32)
    r2 = np.ascontiguousarray(r2, dtype=np.float64)
    return lib().oracle_max_violation(_d(z), z.shape[0], z.shape[1], _i(sides), len(sides),
                                      _d(r2))


def kkt(x0, z, incs, sides, r2, slack=1e-9):
    """KKT certificate; returns dict (see oracle_kkt in smre_oracle.c)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    incs = np.ascontiguousarray(incs, dtype=np.float64)
    sides = np.ascontiguousarray(sides, dtype=np.int32)
    r2 = np.ascontiguousarray(r2, dtype=np.float64)
    out = np.zeros(6)
    rc = lib().oracle_kkt(_d(x0), _d(z), _d(incs), z.shape[0], z.shape[1], _i(sides),
                          len(sides), _d(r2), float(slack), _d(out))
    if rc != 0:
        raise ValueError("oracle_kkt rejected its arguments")
    keys = ["max_violation", "sum_invariant", "mult_residual", "mu_min", "inactive_inc",
            "mu_max"]
    return dict(zip(keys, out.tolist()))


def icd(x0, K, r2, tol=1e-13, mode=TOL_MAXABS, max_inner=100000, num_phases=None):
    """Incomplete Dykstra in FP64.  r2[k] bounds squares of side 2^k, k=0..K.

    Returns (z, total_inner_sweeps).
    """
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    H, W = x0.shape
    r2 = np.ascontiguousarray(r2, dtype=np.float64)
    if len(r2) != K + 1:
        raise ValueError("need K+1 bounds")
    if num_phases is None:
        num_phases = K + 1
    z = np.empty_like(x0)
    tot = ctypes.c_int64(0)
    rc = lib().oracle_icd(_d(x0), H, W, int(K), _d(r2), float(tol), int(mode), int(max_inner),
                          int(num_phases), _d(z), ctypes.byref(tot))
    if rc != 0:
        raise ValueError("oracle_icd rejected its arguments")
    return z, tot.value


# ---------------------------------------------------------------- Monte-Carlo weights

def philox4x64_10(ctr, key):
    """One Philox4x64-10 block: 4 counter words, 2 key words -> 4 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib().oracle_philox4x64_10(c.ctypes.data_as(u64p), k.ctypes.data_as(u64p),
                               out.ctypes.data_as(u64p))
    return out


def mc_field(seed, f, H, W):
    """Field f (H x W) of the Monte-Carlo sample drawn with `seed`."""
    out = np.empty((H, W), dtype=np.float64)
    lib().oracle_mc_field(int(seed), int(f), int(H), int(W), _d(out))
    return out


def mc_statistic(e, sides):
    """(Q, tmax) of one field: Q = max over windows of ((t)^(1/4) - mu_s) / sigma_s,
    tmax[k] = largest window sum of squares of side sides[k]."""
    e = np.ascontiguousarray(e, dtype=np.float64)
    sides = np.ascontiguousarray(sides, dtype=np.int32)
    tmax = np.empty(len(sides), dtype=np.float64)
    q = lib().oracle_mc_statistic(_d(e), e.shape[0], e.shape[1], _i(sides), len(sides),
                                  _d(tmax))
    return q, tmax


def order_quantile(q, alpha):
    """ceil(alpha n)-th smallest of the samples q."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    return lib().oracle_order_quantile(_d(q), len(q), float(alpha))


def icd_family(x0, K, r2, phases, tol=1e-13, mode=TOL_MAXABS, max_inner=100000):
    """ICD over a caller-given phase family: phases = [(shift_y, shift_x,
    min_level), ...].  Returns (z, total_inner_sweeps)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    H, W = x0.shape
    r2 = np.ascontiguousarray(r2, dtype=np.float64)
    if len(r2) != K + 1:
        raise ValueError("need K+1 bounds")
    sy = np.ascontiguousarray([p[0] for p in phases], dtype=np.int32)
    sx = np.ascontiguousarray([p[1] for p in phases], dtype=np.int32)
    lo = np.ascontiguousarray([p[2] for p in phases], dtype=np.int32)
    z = np.empty_like(x0)
    tot = ctypes.c_int64(0)
    rc = lib().oracle_icd_family(_d(x0), H, W, int(K), _d(r2), float(tol), int(mode),
                                 int(max_inner), len(phases), _i(sy), _i(sx), _i(lo), _d(z),
                                 ctypes.byref(tot))
    if rc != 0:
        raise ValueError("oracle_icd_family rejected its arguments")
    return z, tot.value


def icd_nested(x0, level_sides, r2, phases, tol=1e-13, mode=TOL_MAXABS, max_inner=100000):
    """ICD over a nested hierarchy of squares: level j has side level_sides[j]
    (ascending, each dividing the next; blocks of the largest side), bound
    r2[j]; phases = [(shift_y, shift_x, min_level), ...].  Returns
    (z, total_inner_sweeps)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    H, W = x0.shape
    ls = np.ascontiguousarray(level_sides, dtype=np.int32)
    r2 = np.ascontiguousarray(r2, dtype=np.float64)
    if len(r2) != len(ls):
        raise ValueError("need one bound per level")
    sy = np.ascontiguousarray([p[0] for p in phases], dtype=np.int32)
    sx = np.ascontiguousarray([p[1] for p in phases], dtype=np.int32)
    lo = np.ascontiguousarray([p[2] for p in phases], dtype=np.int32)
    z = np.empty_like(x0)
    tot = ctypes.c_int64(0)
    rc = lib().oracle_icd_nested(_d(x0), H, W, len(ls), _i(ls), _d(r2), float(tol), int(mode),
                                 int(max_inner), len(phases), _i(sy), _i(sx), _i(lo), _d(z),
                                 ctypes.byref(tot))
    if rc != 0:
        raise ValueError("oracle_icd_nested rejected its arguments")
    return z, tot.value


def icd_paper_phases(K, num_phases=None):
    """The paper's family: phase i shifted by 2^i mod 2^K on both axes, levels K..i."""
    B = 1 << K
    n = K + 1 if num_phases is None else num_phases
    return [((1 << i) % B, (1 << i) % B, i) for i in range(n)]
