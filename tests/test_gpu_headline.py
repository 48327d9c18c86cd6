"""GPU parity of the headline sweep configuration: FP32 images, window sides
1..16 at region side R = 16 (the kernel instance the 1024^2 benchmark runs),
sides above 17 at R = 32, and BF16-stored increments.

* Per sweep in the same visiting order (region order, same R): FP32 within
  1e-5 of max|z| of the FP64 oracle fed the float32-rounded input, with and
  without the compensated window sums.
* Converged: FP32 at a tight tolerance within 1e-5 of the oracle's limit in
  the canonical order (sides descending, offsets raster), which does not
  depend on the visiting order (Sec. 2.3).
* BF16 increments: the first sweep reads only zero increments, so it equals
  the FP32 sweep bit for bit; the second sweep reads rounded increments, and
  since each window step is nonexpansive in the 2-norm, the two runs differ by
  at most the summed rounding error of the increments read,
  sum_S ||I_S - bf16(I_S)||_2 <= 2^-8 sum_S ||I_S||_2 (I_S the oracle's
  increments after sweep 1).  The converged BF16 error against the oracle is
  printed and gated as stated in the test.
"""
import numpy as np
import pytest

import oracle
import smre_inputs as gi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIDES16 = list(range(1, 17))


@pytest.fixture(scope="module")
def smre():
    import paper_1503_03492_amd as m
    assert torch.cuda.is_available()
    return m


@pytest.fixture(scope="module")
def ctx(smre):
    c = smre.Context(0)
    yield c
    c.close()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def f32_input(H, W, seed):
    # emitter density of the 1024^2 workload (2000 per 1024^2)
    n_e = max(3, round(H * W * 2000 / 1024 ** 2))
    return gi.emitters(H, W, n_e=n_e, seed=seed).astype(np.float32).astype(np.float64)


def gpu_run(ctx, x0, sides, r2, dtype=torch.float32, **opts):
    x = torch.from_numpy(np.ascontiguousarray(x0)).to("cuda", dtype=dtype)
    rc, rep = ctx.project(x, sides, r2, **opts)
    torch.cuda.synchronize()
    return x.double().cpu().numpy(), rc, rep


@pytest.mark.parametrize("H,W,seed", [(96, 112, 1), (97, 113, 2), (50, 130, 3)])
@pytest.mark.parametrize("sweeps", [2, 3])
@pytest.mark.parametrize("kahan", [1, 0])
def test_fp32_sides1_16_per_sweep(ctx, H, W, seed, sweeps, kahan):
    x0 = f32_input(H, W, seed)
    r2 = oracle.chi2_bounds(SIDES16)
    ref, _, _ = oracle.dykstra(x0, SIDES16, r2, tol=0, max_sweeps=sweeps,
                               order=oracle.ORDER_REGION, region=16)
    z, _, rep = gpu_run(ctx, x0, SIDES16, r2, tol=0, max_sweeps=sweeps, region=16, kahan=kahan)
    assert rep["region"] == 16 and rep["sweeps"] == sweeps
    err = relerr(z, ref)
    print(f"FP32 sides 1..16 R=16 {H}x{W} sweeps={sweeps} kahan={kahan}: {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("H,W,sides", [
    (100, 90, [1, 2, 3, 5, 8, 13, 17, 20, 24, 31]),
    (70, 75, SIDES16 + [17, 21, 32]),
])
def test_fp32_r32_per_sweep(ctx, H, W, sides):
    x0 = f32_input(H, W, 4)
    r2 = oracle.chi2_bounds(sides)
    ref, _, _ = oracle.dykstra(x0, sides, r2, tol=0, max_sweeps=2, order=oracle.ORDER_REGION,
                               region=32)
    z, _, rep = gpu_run(ctx, x0, sides, r2, tol=0, max_sweeps=2, region=32)
    assert rep["region"] == 32
    err = relerr(z, ref)
    print(f"FP32 R=32 {H}x{W} sides {sides}: {err:.3e}")
    assert err <= 1e-5


def test_fp32_sides1_16_converged(ctx):
    """Tight FP32 tolerance against the oracle's limit in the canonical order."""
    H, W = 64, 72
    x0 = gi.emitters(H, W, n_e=9, seed=7).astype(np.float32).astype(np.float64)
    r2 = oracle.chi2_bounds(SIDES16)
    try:
        oracle.set_threads(8)
        ref, _, d = oracle.dykstra(x0, SIDES16, r2, tol=1e-11, max_sweeps=100000,
                                   order=oracle.ORDER_DESC)
    finally:
        oracle.set_threads(1)
    assert d < 1e-11
    z, rc, rep = gpu_run(ctx, x0, SIDES16, r2, tol=2e-7, max_sweeps=100000, region=16)
    err = relerr(z, ref)
    print(f"FP32 converged sides 1..16: sweeps {rep['sweeps']}, error {err:.3e}, "
          f"violation {rep['max_violation']:.3e}")
    assert rep["converged"] == 1
    assert err <= 1e-5


def _window_norm_sum(incs, H, W, sides):
    """sum over every window S of ||I_S||_2 from the oracle's canonical layout."""
    tot = 0.0
    t = 0
    for s in sorted(sides, reverse=True):
        for a in range(s):
            for b in range(s):
                plane = incs[t]
                t += 1
                nr, nc = (H - a) // s, (W - b) // s
                if nr <= 0 or nc <= 0:
                    continue
                blk = plane[a:a + nr * s, b:b + nc * s].reshape(nr, s, nc, s)
                tot += float(np.sum(np.sqrt(np.sum(blk * blk, axis=(1, 3)))))
    return tot


@pytest.mark.parametrize("H,W,seed", [(96, 112, 1), (61, 77, 5)])
def test_bf16_first_sweep_equals_fp32_bitwise(ctx, smre, H, W, seed):
    x0 = f32_input(H, W, seed)
    r2 = oracle.chi2_bounds(SIDES16)
    a, _, _ = gpu_run(ctx, x0, SIDES16, r2, tol=0, max_sweeps=1, region=16)
    b, _, _ = gpu_run(ctx, x0, SIDES16, r2, tol=0, max_sweeps=1, region=16, inc=smre.INC_BF16)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("H,W,seed", [(96, 112, 1), (61, 77, 5)])
def test_bf16_second_sweep_within_rounding_bound(ctx, smre, H, W, seed):
    x0 = f32_input(H, W, seed)
    r2 = oracle.chi2_bounds(SIDES16)
    _, _, _, incs = oracle.dykstra(x0, SIDES16, r2, tol=0, max_sweeps=1,
                                   order=oracle.ORDER_REGION, region=16, want_incs=True)
    a, _, _ = gpu_run(ctx, x0, SIDES16, r2, tol=0, max_sweeps=2, region=16)
    b, _, _ = gpu_run(ctx, x0, SIDES16, r2, tol=0, max_sweeps=2, region=16, inc=smre.INC_BF16)
    diff = float(np.sqrt(np.sum((a - b) ** 2)))
    # 2^-8: half an ulp of an 8-bit significand, relative; 1e-3 covers the
    # FP32 increments differing from the oracle's by rounding
    bound = 2.0 ** -8 * _window_norm_sum(incs, H, W, SIDES16) * (1 + 1e-3)
    print(f"BF16 vs FP32 after 2 sweeps {H}x{W}: ||diff||_2 = {diff:.3e}, bound {bound:.3e}")
    assert 0 < diff <= bound


def test_bf16_converged_error_reported(ctx, smre):
    """Converged BF16 run against the oracle's limit.  Every increment store
    rounds to 8 significant bits, which moves the invariant x + sum_S I_S = x0
    by up to 2^-8 |I_S| at the pixels of S; the run settles on the projection
    P(x0 + E) of an input perturbed by the accumulated rounding E, and P is
    nonexpansive.  At the limit all increments at a pixel share one sign, so
    sum_S |I_S,i| = |x0_i - z*_i|: one rounding of every increment moves a
    pixel by at most 2^-8 |x0_i - z*_i|.  The stores repeat every sweep, so E
    is a sum of such roundings; the gate allows four of them, relative to
    max|z*| (measured: about 1.2 on this image, printed)."""
    H, W = 64, 72
    x0 = gi.emitters(H, W, n_e=9, seed=7).astype(np.float32).astype(np.float64)
    r2 = oracle.chi2_bounds(SIDES16)
    try:
        oracle.set_threads(8)
        ref, _, _, incs = oracle.dykstra(x0, SIDES16, r2, tol=1e-11, max_sweeps=100000,
                                         order=oracle.ORDER_DESC, want_incs=True)
    finally:
        oracle.set_threads(1)
    z32, _, rep32 = gpu_run(ctx, x0, SIDES16, r2, tol=1e-5, max_sweeps=100000, region=16)
    zb, _, repb = gpu_run(ctx, x0, SIDES16, r2, tol=1e-5, max_sweeps=100000, region=16,
                          inc=smre.INC_BF16)
    err32, errb = relerr(z32, ref), relerr(zb, ref)
    imax = float(np.max(np.abs(incs)))
    print(f"tol 1e-5: FP32 error {err32:.3e} ({rep32['sweeps']} sweeps), BF16 error "
          f"{errb:.3e} ({repb['sweeps']} sweeps, violation {repb['max_violation']:.3e}); "
          f"max |I| of the limit {imax:.3f}")
    one = 2.0 ** -8 * float(np.max(np.abs(x0 - ref))) / float(np.max(np.abs(ref)))
    print(f"BF16 error in single roundings of the largest total increment: {errb / one:.2f}")
    assert repb["converged"] == 1
    assert errb <= 4 * one
