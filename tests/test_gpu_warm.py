"""GPU parity of warm-started Dykstra (increments kept in the workspace from
the previous solve of the same problem) against the oracle's warm start
(oracle_dykstra_warm: x = x0 - sum_S I_S from the given increments).

Dykstra minimises the dual function of the projection block by block, so it
reaches the same limit from any increments; Algorithm 1 projects a slowly
moving point every iteration (Sec. 2.2), which is what the warm start serves.
"""
import numpy as np
import pytest

import oracle
import oracle.admm as ad
import smre_inputs as gi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smre():
    import paper_1503_03492_amd as m
    assert torch.cuda.is_available()
    return m


@pytest.fixture()
def ctx(smre):
    c = smre.Context(0)
    yield c
    c.close()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu(ctx, x0, sides, r2, dtype=torch.float64, **opts):
    x = torch.from_numpy(np.ascontiguousarray(x0)).to("cuda", dtype=dtype)
    rc, rep = ctx.project(x, sides, r2, **opts)
    torch.cuda.synchronize()
    return x.double().cpu().numpy(), rc, rep


def pair(H, W, seed):
    a = gi.emitters(H, W, n_e=max(3, H * W // 400), seed=seed)
    b = a + 0.05 * gi.gaussian(H, W, seed=seed + 100)
    return a, b


@pytest.mark.parametrize("H,W,sides,R", [(70, 45, list(range(1, 9)), 16),
                                         (41, 96, [1, 2, 4, 7, 12, 16], 16),
                                         (37, 53, [1, 2, 3, 5], 8)])
def test_warm_per_sweep_matches_oracle_fp64(ctx, H, W, sides, R):
    xa, xb = pair(H, W, H + W)
    r2 = oracle.chi2_bounds(sides)
    _, _, _, ia = oracle.dykstra(xa, sides, r2, tol=0, max_sweeps=3, order=oracle.ORDER_REGION,
                                 region=R, want_incs=True)
    ref, _, _ = oracle.dykstra(xb, sides, r2, tol=0, max_sweeps=2, order=oracle.ORDER_REGION,
                               region=R, incs0=ia)
    gpu(ctx, xa, sides, r2, tol=0, max_sweeps=3, region=R)
    z, _, rep = gpu(ctx, xb, sides, r2, tol=0, max_sweeps=2, region=R, warm=True)
    assert rep["sweeps"] == 2
    assert relerr(z, ref) <= 1e-12


def test_warm_per_sweep_fp32(ctx):
    H, W, sides = 96, 112, list(range(1, 17))
    xa, xb = pair(H, W, 3)
    xa = xa.astype(np.float32).astype(np.float64)
    xb = xb.astype(np.float32).astype(np.float64)
    r2 = oracle.chi2_bounds(sides)
    _, _, _, ia = oracle.dykstra(xa, sides, r2, tol=0, max_sweeps=2, order=oracle.ORDER_REGION,
                                 region=16, want_incs=True)
    ref, _, _ = oracle.dykstra(xb, sides, r2, tol=0, max_sweeps=2, order=oracle.ORDER_REGION,
                               region=16, incs0=ia)
    gpu(ctx, xa, sides, r2, dtype=torch.float32, tol=0, max_sweeps=2, region=16)
    z, _, _ = gpu(ctx, xb, sides, r2, dtype=torch.float32, tol=0, max_sweeps=2, region=16,
                  warm=True)
    err = relerr(z, ref)
    print(f"FP32 warm start, sides 1..16: {err:.3e}")
    assert err <= 1e-5


def test_warm_from_own_limit_stops_in_one_sweep(ctx):
    x0 = gi.emitters(48, 52, n_e=6, seed=11)
    sides = [1, 2, 3, 5, 8]
    r2 = oracle.chi2_bounds(sides)
    z1, rc, rep1 = gpu(ctx, x0, sides, r2, tol=1e-13, max_sweeps=100000)
    assert rc == 0
    z2, rc, rep2 = gpu(ctx, x0, sides, r2, tol=1e-12, max_sweeps=100000, warm=True)
    assert rc == 0 and rep2["sweeps"] == 1
    assert relerr(z2, z1) <= 1e-11


def test_warm_converges_to_cold_limit_in_fewer_sweeps(ctx):
    xa, xb = pair(64, 72, 5)
    sides = list(range(1, 9))
    r2 = oracle.chi2_bounds(sides)
    cold, _, rc_ = gpu(ctx, xb, sides, r2, tol=1e-12, max_sweeps=100000)
    gpu(ctx, xa, sides, r2, tol=1e-12, max_sweeps=100000)
    warm, _, rw = gpu(ctx, xb, sides, r2, tol=1e-12, max_sweeps=100000, warm=True)
    print(f"cold {rc_['sweeps']} sweeps, warm {rw['sweeps']} sweeps")
    assert rw["sweeps"] < rc_["sweeps"]
    assert relerr(warm, cold) <= 1e-9


def test_warm_needs_matching_problem(ctx, smre):
    x0 = gi.emitters(40, 44, n_e=5, seed=2)
    sides = [1, 2, 3]
    r2 = oracle.chi2_bounds(sides)
    with pytest.raises(smre.SmreError) as e:  # nothing solved in this context yet
        gpu(ctx, x0, sides, r2, tol=0, max_sweeps=2, warm=True)
    assert e.value.code == -1
    gpu(ctx, x0, sides, r2, tol=0, max_sweeps=2)
    for s2, shape in (([1, 2, 4], (40, 44)), (sides, (40, 45))):
        x1 = gi.emitters(*shape, n_e=5, seed=3)
        with pytest.raises(smre.SmreError):
            gpu(ctx, x1, s2, oracle.chi2_bounds(s2), tol=0, max_sweeps=2, warm=True)
    with pytest.raises(smre.SmreError):  # other bounds
        gpu(ctx, x0, sides, r2 * 1.01, tol=0, max_sweeps=2, warm=True)
    with pytest.raises(smre.SmreError):  # other precision
        gpu(ctx, x0, sides, r2, dtype=torch.float32, tol=0, max_sweeps=2, warm=True)


def test_admm_full_warm_matches_oracle_and_saves_sweeps(ctx, smre):
    H, W, sigma, sides, iters = 16, 18, 1.0, [1, 2, 3], 12
    I = gi.gaussian(H, W, seed=4, scale=2.0)
    r2 = oracle.chi2_bounds(sides)
    ref = ad.admm(I, sigma, lambda X: ad.project_full(X, sides, r2, 1e-14), delta=-1.0,
                  max_iter=iters)
    kw = dict(method=smre.ADMM_FULL, sides=sides, radius2=r2, full_tol=1e-14,
              full_max_sweeps=100000, delta=-1.0, max_iter=iters, want_eps=True)
    Id = torch.from_numpy(I).cuda()
    xc, ec, rc_ = ctx.admm(Id, sigma, **kw)
    xw, ew, rw = ctx.admm(Id, sigma, full_warm=True, **kw)
    print(f"ADMM exact projections: cold {rc_['projection_sweeps']} sweeps, "
          f"warm {rw['projection_sweeps']}")
    assert rw["projection_sweeps"] < rc_["projection_sweeps"]
    assert relerr(xw.cpu().numpy(), ref["x"]) <= 1e-9
    assert relerr(ew.cpu().numpy(), ref["eps"]) <= 1e-9
