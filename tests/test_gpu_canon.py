"""GPU parity of full Dykstra in the canonical visiting orders (sides
descending or ascending, each side's tilings (a, b) in raster order; one
launch per tiling) against the oracle in the same order.

* Per sweep, FP64: within 1e-12 of max|z| -- the same sets in the same order,
  so only the summation order inside a window differs.
* Per sweep, FP32 on the float32-rounded input: within 1e-5.
* Converged: the canonical-order limit equals the region-order limit (Sec.
  2.3: the limit does not depend on the cyclic order).
* BF16 increments: the first sweep reads only zeros, so it equals FP32 bit for
  bit.
* Warm start keeps the order in the problem signature.
"""
import numpy as np
import pytest

import oracle
import smre_inputs as gi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def gpu_run(ctx, x0, sides, r2, dtype=torch.float64, **opts):
    x = torch.from_numpy(np.ascontiguousarray(x0)).to("cuda", dtype=dtype)
    rc, rep = ctx.project(x, sides, r2, **opts)
    torch.cuda.synchronize()
    return x.double().cpu().numpy(), rc, rep


def orders(smre):
    return [(smre.ORDER_DESC, oracle.ORDER_DESC), (smre.ORDER_ASC, oracle.ORDER_ASC)]


@pytest.mark.parametrize("H,W,sides", [
    (37, 53, [1, 2, 3, 5]),
    (70, 45, list(range(1, 9))),
    (41, 96, [1, 2, 4, 7, 12, 16, 17, 25, 32]),
    (1, 33, [1]),
    (33, 1, [1]),
])
@pytest.mark.parametrize("which", [0, 1])
def test_fp64_per_sweep(ctx, smre, H, W, sides, which):
    lib_order, or_order = orders(smre)[which]
    x0 = gi.emitters(H, W, n_e=max(3, H * W // 300), seed=H * W)
    r2 = oracle.chi2_bounds(sides)
    for sweeps in (1, 3):
        ref, _, _ = oracle.dykstra(x0, sides, r2, tol=0, max_sweeps=sweeps, order=or_order)
        z, rc, rep = gpu_run(ctx, x0, sides, r2, tol=0, max_sweeps=sweeps, order=lib_order)
        assert rc == 0 and rep["sweeps"] == sweeps
        assert relerr(z, ref) <= 1e-12, (sweeps, relerr(z, ref))


@pytest.mark.parametrize("H,W,sides", [(96, 112, list(range(1, 17))),
                                       (97, 113, list(range(1, 17))),
                                       (70, 75, [1, 2, 3, 8, 16, 17, 21, 32])])
@pytest.mark.parametrize("kahan", [1, 0])
def test_fp32_per_sweep(ctx, smre, H, W, sides, kahan):
    n_e = max(3, round(H * W * 2000 / 1024 ** 2))
    x0 = gi.emitters(H, W, n_e=n_e, seed=9).astype(np.float32).astype(np.float64)
    r2 = oracle.chi2_bounds(sides)
    ref, _, _ = oracle.dykstra(x0, sides, r2, tol=0, max_sweeps=3, order=oracle.ORDER_DESC)
    z, _, _ = gpu_run(ctx, x0, sides, r2, dtype=torch.float32, tol=0, max_sweeps=3,
                      order=smre.ORDER_DESC, kahan=kahan)
    err = relerr(z, ref)
    print(f"FP32 canonical order {H}x{W} kahan={kahan}: {err:.3e}")
    assert err <= 1e-5


def test_converged_matches_region_order_limit(ctx, smre):
    x0 = gi.emitters(48, 52, n_e=6, seed=12)
    sides = [1, 2, 3, 5, 8]
    r2 = oracle.chi2_bounds(sides)
    ref, ks, _ = oracle.dykstra(x0, sides, r2, tol=1e-12, max_sweeps=100000,
                                order=oracle.ORDER_DESC)
    zc, rc, rep = gpu_run(ctx, x0, sides, r2, tol=1e-12, max_sweeps=100000,
                          order=smre.ORDER_DESC)
    zr, rr, _ = gpu_run(ctx, x0, sides, r2, tol=1e-13, max_sweeps=100000)
    print(f"canonical: {rep['sweeps']} sweeps (oracle {ks}); violation {rep['max_violation']:.2e}")
    assert rc == 0 and rr == 0 and rep["converged"] == 1
    assert abs(rep["sweeps"] - ks) <= 1
    assert relerr(zc, ref) <= 1e-10
    assert relerr(zc, zr) <= 1e-9


@pytest.mark.parametrize("H,W", [(96, 112), (61, 77)])
def test_bf16_first_sweep_equals_fp32(ctx, smre, H, W):
    x0 = gi.emitters(H, W, n_e=8, seed=3).astype(np.float32).astype(np.float64)
    sides = list(range(1, 17))
    r2 = oracle.chi2_bounds(sides)
    a, _, _ = gpu_run(ctx, x0, sides, r2, dtype=torch.float32, tol=0, max_sweeps=1,
                      order=smre.ORDER_DESC)
    b, _, _ = gpu_run(ctx, x0, sides, r2, dtype=torch.float32, tol=0, max_sweeps=1,
                      order=smre.ORDER_DESC, inc=smre.INC_BF16)
    assert np.array_equal(a, b)


def test_warm_start_in_canonical_order(ctx, smre):
    H, W = 40, 44
    xa = gi.emitters(H, W, n_e=5, seed=21)
    xb = xa + 0.05 * gi.gaussian(H, W, seed=22)
    sides = [1, 2, 3, 6]
    r2 = oracle.chi2_bounds(sides)
    _, _, _, ia = oracle.dykstra(xa, sides, r2, tol=0, max_sweeps=3, order=oracle.ORDER_ASC,
                                 want_incs=True)
    ref, _, _ = oracle.dykstra(xb, sides, r2, tol=0, max_sweeps=2, order=oracle.ORDER_ASC,
                               incs0=ia)
    gpu_run(ctx, xa, sides, r2, tol=0, max_sweeps=3, order=smre.ORDER_ASC)
    z, _, rep = gpu_run(ctx, xb, sides, r2, tol=0, max_sweeps=2, order=smre.ORDER_ASC, warm=True)
    assert rep["sweeps"] == 2
    assert relerr(z, ref) <= 1e-12
    # increments left by another order are not this problem's
    with pytest.raises(smre.SmreError):
        gpu_run(ctx, xb, sides, r2, tol=0, max_sweeps=2, order=smre.ORDER_DESC, warm=True)


def test_invalid_order_rejected(ctx, smre):
    x0 = gi.emitters(20, 20, n_e=3, seed=1)
    for bad in (3, -1):
        with pytest.raises(smre.SmreError) as e:
            gpu_run(ctx, x0, [1, 2], oracle.chi2_bounds([1, 2]), tol=0, max_sweeps=1, order=bad)
        assert e.value.code == -1
