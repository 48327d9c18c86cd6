"""Python binding of libsmre.so (the MI355X SMRE projection library).

Argument marshalling only: every step of the projection runs in the HIP
kernels behind the C ABI declared in include/smre.h.  PyTorch supplies device
memory and the current stream.  There is no CPU fallback: if the library is
missing, importing this package raises.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmre.so")

OK = 0
NOT_CONVERGED = 1
PENDING = 2
F32, F64 = 0, 1
INC_SAME, INC_BF16 = 0, 1
ORDER_REGION, ORDER_DESC, ORDER_ASC = 0, 1, 2
TOL_MAXABS, TOL_MEANABS = 0, 1


class SmreError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {status_string(code)} ({code})")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("n_sides", ctypes.c_int32), ("sides", ctypes.POINTER(ctypes.c_int32)),
                ("radius2", ctypes.POINTER(ctypes.c_double)), ("tol", ctypes.c_double),
                ("max_sweeps", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("region", ctypes.c_int32), ("inc", ctypes.c_int32), ("kahan", ctypes.c_int32),
                ("warm", ctypes.c_int32), ("guard_rel", ctypes.c_double),
                ("order", ctypes.c_int32), ("reserved1", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("region", ctypes.c_int32), ("inner_sweeps", ctypes.c_int32),
                ("last_delta", ctypes.c_double), ("max_violation", ctypes.c_double),
                ("elapsed_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("bytes_moved", ctypes.c_double), ("window_projections", ctypes.c_double),
                ("kernel_launches", ctypes.c_int64), ("pixel_updates", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchImage(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("H", ctypes.c_int64), ("W", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("n_sides", ctypes.c_int32),
                ("sides", ctypes.POINTER(ctypes.c_int32)),
                ("radius2", ctypes.POINTER(ctypes.c_double)), ("tol", ctypes.c_double),
                ("max_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchParams(ctypes.Structure):
    _fields_ = [("region", ctypes.c_int32), ("inc", ctypes.c_int32), ("kahan", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("guard_rel", ctypes.c_double),
                ("use_graph", ctypes.c_int32), ("grid", ctypes.c_int32)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_size_t),
                ("max_active", ctypes.c_int32), ("queue_cap", ctypes.c_int32),
                ("inc", ctypes.c_int32), ("kahan", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("guard_rel", ctypes.c_double)]


class ServeCounters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "rejected", "failed",
                                              "active", "queued", "sweeps", "bytes_in_use",
                                              "peak_active", "joined_running")]


class AdmmParams(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("lam", ctypes.c_double), ("rho1", ctypes.c_double),
                ("rho2", ctypes.c_double), ("alpha1", ctypes.c_double),
                ("alpha2", ctypes.c_double), ("gamma", ctypes.c_double),
                ("delta", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("method", ctypes.c_int32), ("K", ctypes.c_int32),
                ("icd_tolmode", ctypes.c_int32), ("icd_tol", ctypes.c_double),
                ("icd_max_inner", ctypes.c_int32), ("warm", ctypes.c_int32),
                ("radius2_icd", ctypes.POINTER(ctypes.c_double)),
                ("full", ctypes.POINTER(Params))]


class AdmmReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("last_dx", ctypes.c_double), ("last_residual", ctypes.c_double),
                ("elapsed_ms", ctypes.c_double), ("projection_ms", ctypes.c_double),
                ("projection_sweeps", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ADMM_ICD, ADMM_FULL = 0, 1


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(or python -m paper_1503_03492_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    ip, dp = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    L.smre_status_string.argtypes = [ctypes.c_int]
    L.smre_status_string.restype = ctypes.c_char_p
    L.smre_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    L.smre_ctx_destroy.argtypes = [vp]
    L.smre_ctx_destroy.restype = None
    L.smre_ctx_set_timing.argtypes = [vp, ctypes.c_int]
    L.smre_chi2_bounds.argtypes = [ip, i32, dbl, dp]
    L.smre_paper_bounds.argtypes = [ip, i32, dbl, dp]
    L.smre_workspace_size.argtypes = [ctypes.c_int, i64, i64, ctypes.POINTER(Params),
                                      ctypes.POINTER(ctypes.c_size_t)]
    L.smre_dykstra_project.argtypes = [vp, ctypes.c_int, vp, i64, i64, i64,
                                       ctypes.POINTER(Params), vp, ctypes.c_size_t, vp,
                                       ctypes.POINTER(Report)]
    L.smre_dykstra_incomplete.argtypes = [vp, ctypes.c_int, vp, i64, i64, i64, i32, dp, dbl,
                                          i32, i32, i32, vp, ctypes.POINTER(Report)]
    L.smre_dykstra_incomplete_noalloc.argtypes = L.smre_dykstra_incomplete.argtypes
    L.smre_dykstra_incomplete_frames.argtypes = [vp, ctypes.c_int, vp, i64, i64, i64, i64, i32,
                                                 dp, dbl, i32, i32, i32, vp,
                                                 ctypes.POINTER(Report)]
    L.smre_dykstra_incomplete_family.argtypes = [vp, ctypes.c_int, vp, i64, i64, i64, i64, i32,
                                                 dp, i32, ip, ip, ip, dbl, i32, i32, vp,
                                                 ctypes.POINTER(Report)]
    L.smre_dykstra_incomplete_nested.argtypes = [vp, ctypes.c_int, vp, i64, i64, i64, i64, i32,
                                                 ip, dp, i32, ip, ip, ip, dbl, i32, i32, vp,
                                                 ctypes.POINTER(Report)]
    L.smre_max_violation.argtypes = [vp, ctypes.c_int, vp, i64, i64, i64, i32, ip, dp, vp, dp]
    L.smre_batch_workspace_size.argtypes = [ctypes.c_int, i32, ctypes.POINTER(BatchImage),
                                            ctypes.POINTER(BatchParams),
                                            ctypes.POINTER(ctypes.c_size_t)]
    L.smre_dykstra_project_batch.argtypes = [vp, ctypes.c_int, i32, ctypes.POINTER(BatchImage),
                                             ctypes.POINTER(BatchParams), vp, ctypes.c_size_t,
                                             vp, ctypes.POINTER(Report)]
    L.smre_serve_create.argtypes = [ctypes.POINTER(ServeConfig), ctypes.POINTER(vp)]
    L.smre_serve_destroy.argtypes = [vp]
    L.smre_serve_destroy.restype = None
    L.smre_serve_submit.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32, i32,
                                    ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_uint64)]
    L.smre_serve_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float),
                                  ctypes.c_size_t, ctypes.POINTER(Report),
                                  ctypes.POINTER(ctypes.c_double)]
    L.smre_serve_stats.argtypes = [vp, ctypes.POINTER(ServeCounters)]
    L.smre_admm.argtypes = [vp, ctypes.c_int, vp, vp, i64, i64, i64, ctypes.POINTER(AdmmParams),
                            vp, vp, ctypes.POINTER(AdmmReport)]
    u64 = ctypes.c_uint64
    L.smre_mc_fields.argtypes = [vp, i64, i64, u64, i64, i64, vp, i64, vp]
    L.smre_mc_statistic.argtypes = [vp, i64, i64, i32, ip, u64, i64, i64, dp, dp, vp,
                                    ctypes.POINTER(Report)]
    L.smre_mc_statistic_fields.argtypes = [vp, ctypes.c_int, vp, i64, i64, i64, i64, i32, ip, dp,
                                           dp, vp]
    L.smre_mc_quantile.argtypes = [vp, i64, i64, i32, ip, u64, i64, dbl, dp, vp,
                                   ctypes.POINTER(Report)]
    return L


_lib = _load()

EXPORTS = ["smre_status_string", "smre_ctx_create", "smre_ctx_destroy", "smre_ctx_set_timing",
           "smre_chi2_bounds", "smre_paper_bounds", "smre_workspace_size",
           "smre_dykstra_project", "smre_dykstra_incomplete", "smre_dykstra_incomplete_frames",
           "smre_dykstra_incomplete_family", "smre_dykstra_incomplete_noalloc",
           "smre_dykstra_incomplete_nested",
           "smre_max_violation",
           "smre_batch_workspace_size", "smre_dykstra_project_batch", "smre_serve_create",
           "smre_serve_destroy", "smre_serve_submit", "smre_serve_poll", "smre_serve_stats",
           "smre_mc_fields", "smre_mc_statistic", "smre_mc_statistic_fields", "smre_mc_quantile",
           "smre_admm"]


def lib():
    return _lib


def status_string(code):
    return _lib.smre_status_string(int(code)).decode()


def _frames(x):
    """(frames, H, W, ld) of a 2-D image or an (n, H, W) stack of frames."""
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dim() not in (2, 3):
        raise TypeError("x must be a 2-D or 3-D CUDA tensor")
    if x.dim() == 2:
        return (1,) + tuple(_image(x))
    if x.stride(2) != 1 or x.stride(0) != x.shape[1] * x.stride(1):
        raise ValueError("frames must be stacked at stride H * ld")
    return x.shape[0], x.shape[1], x.shape[2], x.stride(1)


def _check(code, what, allow=(OK,)):
    if code not in allow:
        raise SmreError(code, what)
    return code


def _ivec(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _dvec(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def chi2_bounds(sides, p=0.9):
    s, sp = _ivec(sides)
    out = np.empty(len(s))
    _check(_lib.smre_chi2_bounds(sp, len(s), float(p), _dvec(out)[1]), "smre_chi2_bounds")
    return out


def paper_bounds(sides, q_alpha):
    s, sp = _ivec(sides)
    out = np.empty(len(s))
    _check(_lib.smre_paper_bounds(sp, len(s), float(q_alpha), _dvec(out)[1]),
           "smre_paper_bounds")
    return out


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("x must be float32 or float64")


def _image(x):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("x must be a CUDA (HIP) tensor")
    if x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("x must be 2-D with unit column stride")
    return x.shape[0], x.shape[1], x.stride(0)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclass
class ProjectOptions:
    tol: float = 1e-5
    max_sweeps: int = 5000
    check_every: int = 1
    region: int = 0
    inc: int = INC_SAME
    kahan: bool = True
    guard_rel: float = 1e-5
    # start from the increments the previous call on the same problem left in
    # the workspace (the context's cached one, or the one passed)
    warm: bool = False
    # cyclic order: ORDER_REGION (default) or the canonical ORDER_DESC / ORDER_ASC
    order: int = ORDER_REGION


class Context:
    """One per device and host thread; caches the workspace between calls."""

    def __init__(self, device=0):
        h = ctypes.c_void_p()
        _check(_lib.smre_ctx_create(int(device), ctypes.byref(h)), "smre_ctx_create")
        self._h = h
        self.device = device

    def close(self):
        if self._h:
            _lib.smre_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, on):
        """on: False / True (every sweep-kernel launch), or k >= 1 (every k-th
        launch of a call)."""
        every = (1 if on else 0) if isinstance(on, bool) else int(on)
        _check(_lib.smre_ctx_set_timing(self._h, every), "smre_ctx_set_timing")

    @staticmethod
    def _params(sides, radius2, o):
        s, sp = _ivec(sides)
        r, rp = _dvec(radius2)
        if len(s) != len(r):
            raise ValueError("sides and radius2 differ in length")
        p = Params(len(s), sp, rp, float(o.tol), int(o.max_sweeps), int(o.check_every),
                   int(o.region), int(o.inc), 1 if o.kahan else 0, 1 if o.warm else 0,
                   float(o.guard_rel), int(o.order), 0)
        return p, (s, r)

    def workspace_size(self, dtype, H, W, sides, radius2, opts=None):
        p, keep = self._params(sides, radius2, opts or ProjectOptions())
        n = ctypes.c_size_t()
        _check(_lib.smre_workspace_size(int(dtype), H, W, ctypes.byref(p), ctypes.byref(n)),
               "smre_workspace_size")
        return n.value

    def project(self, x, sides, radius2, opts=None, workspace=None, stream=None, **kw):
        """Full Dykstra projection of x (2-D CUDA tensor), in place.  Returns
        (status, report dict); status is OK or NOT_CONVERGED."""
        o = opts or ProjectOptions()
        for k, v in kw.items():
            setattr(o, k, v)
        H, W, ld = _image(x)
        p, keep = self._params(sides, radius2, o)
        rep = Report()
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            ws_ptr, ws_bytes = ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * \
                workspace.element_size()
        rc = _lib.smre_dykstra_project(self._h, _dtype_code(x), ctypes.c_void_p(x.data_ptr()), H,
                                       W, ld, ctypes.byref(p), ws_ptr, ws_bytes,
                                       _stream(stream), ctypes.byref(rep))
        _check(rc, "smre_dykstra_project", allow=(OK, NOT_CONVERGED))
        return rc, rep.as_dict()

    def incomplete(self, x, K, radius2, tol=1e-3, mode=TOL_MEANABS, max_inner=10000,
                   num_phases=None, stream=None):
        """Incomplete Dykstra of x (2-D CUDA tensor), in place; returns report dict."""
        H, W, ld = _image(x)
        r, rp = _dvec(radius2)
        if len(r) != K + 1:
            raise ValueError("radius2 needs K+1 entries")
        if num_phases is None:
            num_phases = K + 1
        rep = Report()
        rc = _lib.smre_dykstra_incomplete(self._h, _dtype_code(x), ctypes.c_void_p(x.data_ptr()),
                                          H, W, ld, int(K), rp, float(tol), int(mode),
                                          int(max_inner), int(num_phases), _stream(stream),
                                          ctypes.byref(rep))
        _check(rc, "smre_dykstra_incomplete", allow=(OK, NOT_CONVERGED))
        return rep.as_dict()

    def incomplete_noalloc(self, x, K, radius2, tol=1e-3, mode=TOL_MEANABS, max_inner=10000,
                           num_phases=None, stream=None):
        """As incomplete(), through the entry point that allocates no device
        memory (its scratch is a fixed static array per GPU; overlapping calls
        on one GPU race)."""
        H, W, ld = _image(x)
        r, rp = _dvec(radius2)
        if len(r) != K + 1:
            raise ValueError("radius2 needs K+1 entries")
        if num_phases is None:
            num_phases = K + 1
        rep = Report()
        rc = _lib.smre_dykstra_incomplete_noalloc(self._h, _dtype_code(x),
                                                  ctypes.c_void_p(x.data_ptr()), H, W, ld, int(K),
                                                  rp, float(tol), int(mode), int(max_inner),
                                                  int(num_phases), _stream(stream),
                                                  ctypes.byref(rep))
        _check(rc, "smre_dykstra_incomplete_noalloc", allow=(OK, NOT_CONVERGED))
        return rep.as_dict()

    def incomplete_frames(self, x, K, radius2, tol=1e-3, mode=TOL_MEANABS, max_inner=10000,
                          num_phases=None, stream=None):
        """Incomplete Dykstra of every frame of x, an (n, H, W) CUDA tensor with
        frames stacked at stride H * ld, in place; returns the report dict."""
        import torch
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dim() != 3:
            raise TypeError("x must be an (n, H, W) CUDA tensor")
        if x.stride(2) != 1 or x.stride(0) != x.shape[1] * x.stride(1):
            raise ValueError("frames must be stacked at stride H * ld with unit column stride")
        n, H, W = x.shape
        r, rp = _dvec(radius2)
        if len(r) != K + 1:
            raise ValueError("radius2 needs K+1 entries")
        if num_phases is None:
            num_phases = K + 1
        rep = Report()
        rc = _lib.smre_dykstra_incomplete_frames(self._h, _dtype_code(x),
                                                 ctypes.c_void_p(x.data_ptr()), H, W, x.stride(1),
                                                 n, int(K), rp, float(tol), int(mode),
                                                 int(max_inner), int(num_phases), _stream(stream),
                                                 ctypes.byref(rep))
        _check(rc, "smre_dykstra_incomplete_frames", allow=(OK, NOT_CONVERGED))
        return rep.as_dict()

    def incomplete_family(self, x, K, radius2, phases, tol=1e-3, mode=TOL_MEANABS,
                          max_inner=10000, stream=None):
        """ICD over a phase family [(shift_y, shift_x, min_level), ...] on x, a 2-D
        image or an (n, H, W) stack of frames (CUDA tensor), in place."""
        n, H, W, ld = _frames(x)
        r, rp = _dvec(radius2)
        if len(r) != K + 1:
            raise ValueError("radius2 needs K+1 entries")
        sy, syp = _ivec([p[0] for p in phases])
        sx, sxp = _ivec([p[1] for p in phases])
        lo, lop = _ivec([p[2] for p in phases])
        rep = Report()
        rc = _lib.smre_dykstra_incomplete_family(self._h, _dtype_code(x),
                                                 ctypes.c_void_p(x.data_ptr()), H, W, ld, n,
                                                 int(K), rp, len(sy), syp, sxp, lop, float(tol),
                                                 int(mode), int(max_inner), _stream(stream),
                                                 ctypes.byref(rep))
        _check(rc, "smre_dykstra_incomplete_family", allow=(OK, NOT_CONVERGED))
        return rep.as_dict()

    def incomplete_nested(self, x, level_sides, radius2, phases, tol=1e-3, mode=TOL_MEANABS,
                          max_inner=10000, stream=None):
        """ICD over a nested hierarchy of squares: level j has side
        level_sides[j] (ascending, each dividing the next) and bound
        radius2[j]; phases = [(shift_y, shift_x, min_level), ...].  x is a 2-D
        image or an (n, H, W) stack of frames (CUDA tensor), in place."""
        n, H, W, ld = _frames(x)
        ls, lsp = _ivec(level_sides)
        r, rp = _dvec(radius2)
        if len(r) != len(ls):
            raise ValueError("radius2 needs one entry per level")
        sy, syp = _ivec([p[0] for p in phases])
        sx, sxp = _ivec([p[1] for p in phases])
        lo, lop = _ivec([p[2] for p in phases])
        rep = Report()
        rc = _lib.smre_dykstra_incomplete_nested(self._h, _dtype_code(x),
                                                 ctypes.c_void_p(x.data_ptr()), H, W, ld, n,
                                                 len(ls), lsp, rp, len(sy), syp, sxp, lop,
                                                 float(tol), int(mode), int(max_inner),
                                                 _stream(stream), ctypes.byref(rep))
        _check(rc, "smre_dykstra_incomplete_nested", allow=(OK, NOT_CONVERGED))
        return rep.as_dict()

    def project_batch(self, xs, sides, radius2, tol=1e-5, max_sweeps=5000, region=0,
                      inc=INC_SAME, kahan=True, check_every=1, guard_rel=1e-5, use_graph=True,
                      grid=0, stream=None):
        """Full Dykstra on a list of 2-D CUDA tensors (same dtype), in place.

        sides / radius2 / tol / max_sweeps may be per-image lists or shared.
        Returns (status, list of report dicts)."""
        n = len(xs)
        if n == 0:
            raise ValueError("empty batch")
        dt = _dtype_code(xs[0])
        per = lambda v: v if (isinstance(v, (list, tuple)) and len(v) == n and
                              hasattr(v[0], "__len__")) else [v] * n
        sides_l, r2_l = per(sides), per(radius2)
        tol_l = tol if isinstance(tol, (list, tuple)) else [tol] * n
        ms_l = max_sweeps if isinstance(max_sweeps, (list, tuple)) else [max_sweeps] * n
        imgs = (BatchImage * n)()
        keep = []
        for i, x in enumerate(xs):
            if _dtype_code(x) != dt:
                raise TypeError("all images need one dtype")
            H, W, ld = _image(x)
            sv, sp = _ivec(sides_l[i])
            rv, rp = _dvec(r2_l[i])
            keep += [sv, rv]
            imgs[i] = BatchImage(x.data_ptr(), H, W, ld, len(sv), sp, rp, float(tol_l[i]),
                                 int(ms_l[i]), 0)
        bp = BatchParams(int(region), int(inc), 1 if kahan else 0, int(check_every),
                         float(guard_rel), 1 if use_graph else 0, int(grid))
        reps = (Report * n)()
        rc = _lib.smre_dykstra_project_batch(self._h, dt, n, imgs, ctypes.byref(bp), None, 0,
                                             _stream(stream), reps)
        _check(rc, "smre_dykstra_project_batch", allow=(OK, NOT_CONVERGED))
        return rc, [r.as_dict() for r in reps]

    def max_violation(self, x, sides, radius2, stream=None):
        H, W, ld = _image(x)
        s, sp = _ivec(sides)
        r, rp = _dvec(radius2)
        out = ctypes.c_double()
        _check(_lib.smre_max_violation(self._h, _dtype_code(x), ctypes.c_void_p(x.data_ptr()), H,
                                       W, ld, len(s), sp, rp, _stream(stream), ctypes.byref(out)),
               "smre_max_violation")
        return out.value

    # ---- ADMM outer loop ----
    def admm(self, I, sigma, method=ADMM_ICD, K=4, radius2_icd=None, icd_tol=1e-3,
             icd_mode=TOL_MEANABS, icd_max_inner=10000, sides=None, radius2=None, full_tol=1e-5,
             full_max_sweeps=5000, lam=1.0, rho1=6.192, rho2=1.8, alpha1=1.2, alpha2=0.12,
             gamma=0.0, delta=1e-3, max_iter=100, want_eps=False, full_warm=False,
             stream=None):
        """ADMM estimate x (new tensor like I) for the data I (2-D CUDA tensor);
        returns (x, report) or (x, eps, report)."""
        import torch
        H, W, ld = _image(I)
        x = torch.empty_strided(I.size(), I.stride(), dtype=I.dtype, device=I.device)
        eps = (torch.empty_strided(I.size(), I.stride(), dtype=I.dtype, device=I.device)
               if want_eps else None)
        keep = []
        p = AdmmParams(float(sigma), float(lam), float(rho1), float(rho2), float(alpha1),
                       float(alpha2), float(gamma), float(delta), int(max_iter), int(method),
                       int(K), int(icd_mode), float(icd_tol), int(icd_max_inner),
                       1 if full_warm else 0, None, None)
        if method == ADMM_ICD:
            r, rp = _dvec(radius2_icd)
            keep.append(r)
            p.radius2_icd = rp
        else:
            s_, sp = _ivec(sides)
            r, rp = _dvec(radius2)
            keep += [s_, r]
            fp = Params(len(s_), sp, rp, float(full_tol), int(full_max_sweeps), 1, 0, INC_SAME,
                        1, 0, 1e-5)
            keep.append(fp)
            p.full = ctypes.pointer(fp)
        rep = AdmmReport()
        _check(_lib.smre_admm(self._h, _dtype_code(I), ctypes.c_void_p(I.data_ptr()),
                              ctypes.c_void_p(x.data_ptr()), H, W, ld, ctypes.byref(p),
                              ctypes.c_void_p(eps.data_ptr()) if eps is not None else None,
                              _stream(stream), ctypes.byref(rep)), "smre_admm")
        if want_eps:
            return x, eps, rep.as_dict()
        return x, rep.as_dict()

    # ---- Monte-Carlo weights (the paper's q_alpha) ----
    def mc_fields(self, out, seed, field0=0, stream=None):
        """Write drawn fields field0 .. field0 + n - 1 into out, a float64 CUDA
        tensor of shape (n, H, W) with unit column stride."""
        import torch
        if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.float64:
            raise TypeError("out must be a float64 CUDA tensor")
        if out.dim() != 3 or out.stride(2) != 1 or out.stride(0) != out.shape[1] * out.stride(1):
            raise ValueError("out must be (n, H, W) with fields stacked at stride H * ld")
        n, H, W = out.shape
        _check(_lib.smre_mc_fields(self._h, H, W, int(seed), int(field0), n,
                                   ctypes.c_void_p(out.data_ptr()), out.stride(1),
                                   _stream(stream)), "smre_mc_fields")

    def mc_statistic(self, H, W, sides, seed, n_fields, field0=0, want_tmax=False, stream=None):
        """Q of drawn fields (numpy array); with want_tmax also the largest
        window sum of squares per (field, side)."""
        s, sp = _ivec(sides)
        q = np.empty(int(n_fields))
        t = np.empty((int(n_fields), len(s))) if want_tmax else None
        rep = Report()
        _check(_lib.smre_mc_statistic(self._h, int(H), int(W), len(s), sp, int(seed), int(field0),
                                      int(n_fields), _dvec(q)[1],
                                      _dvec(t)[1] if t is not None else None, _stream(stream),
                                      ctypes.byref(rep)), "smre_mc_statistic")
        return (q, t, rep.as_dict()) if want_tmax else (q, rep.as_dict())

    def mc_statistic_fields(self, fields, sides, stream=None):
        """(Q, tmax) of caller-supplied fields: a (n, H, W) CUDA tensor."""
        import torch
        if not isinstance(fields, torch.Tensor) or not fields.is_cuda or fields.dim() != 3:
            raise TypeError("fields must be an (n, H, W) CUDA tensor")
        if fields.stride(2) != 1 or fields.stride(0) != fields.shape[1] * fields.stride(1):
            raise ValueError("fields must be stacked at stride H * ld with unit column stride")
        n, H, W = fields.shape
        s, sp = _ivec(sides)
        q = np.empty(n)
        t = np.empty((n, len(s)))
        _check(_lib.smre_mc_statistic_fields(self._h, _dtype_code(fields),
                                             ctypes.c_void_p(fields.data_ptr()), H, W,
                                             fields.stride(1), n, len(s), sp, _dvec(q)[1],
                                             _dvec(t)[1], _stream(stream)),
               "smre_mc_statistic_fields")
        return q, t

    def mc_quantile(self, H, W, sides, seed, n_fields, alpha, stream=None):
        """(q_alpha, report) from fields 0 .. n_fields - 1."""
        s, sp = _ivec(sides)
        q = ctypes.c_double()
        rep = Report()
        _check(_lib.smre_mc_quantile(self._h, int(H), int(W), len(s), sp, int(seed),
                                     int(n_fields), float(alpha), ctypes.byref(q),
                                     _stream(stream), ctypes.byref(rep)), "smre_mc_quantile")
        return q.value, rep.as_dict()


class Server:
    """Continuous-batching projection server (FP32 images, host in / host out)."""

    def __init__(self, device=0, hbm_budget_bytes=0, max_active=16, queue_cap=1024,
                 inc=INC_SAME, kahan=True, check_every=1, guard_rel=1e-5):
        cfg = ServeConfig(int(device), int(hbm_budget_bytes), int(max_active), int(queue_cap),
                          int(inc), 1 if kahan else 0, int(check_every), 0, float(guard_rel))
        h = ctypes.c_void_p()
        _check(_lib.smre_serve_create(ctypes.byref(cfg), ctypes.byref(h)), "smre_serve_create")
        self._h = h

    def close(self):
        if self._h:
            _lib.smre_serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, x, sides, radius2, tol=1e-5, max_sweeps=5000):
        """x: 2-D float32 numpy array.  Returns a ticket (int) or raises SmreError."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        s, sp = _ivec(sides)
        r, rp = _dvec(radius2)
        p = Params(len(s), sp, rp, float(tol), int(max_sweeps), 1, 16, 0, 1, 0, 0.0)
        t = ctypes.c_uint64()
        _check(_lib.smre_serve_submit(self._h, x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                      x.shape[0], x.shape[1], ctypes.byref(p), ctypes.byref(t)),
               "smre_serve_submit")
        return t.value

    def poll(self, ticket, shape):
        """None while pending; else (status, result array, report dict, latency s)."""
        out = np.empty(shape, dtype=np.float32)
        rep = Report()
        lat = ctypes.c_double()
        rc = _lib.smre_serve_poll(self._h, ctypes.c_uint64(ticket),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), out.size,
                                  ctypes.byref(rep), ctypes.byref(lat))
        if rc == PENDING:
            return None
        return rc, out, rep.as_dict(), lat.value

    def stats(self):
        c = ServeCounters()
        _check(_lib.smre_serve_stats(self._h, ctypes.byref(c)), "smre_serve_stats")
        return {k: getattr(c, k) for k, _ in c._fields_}
