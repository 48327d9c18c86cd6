"""GPU parity of the nested-hierarchy ICD (smre_dykstra_incomplete_nested, and
smre_dykstra_incomplete with K = 6) against oracle_icd_nested.

Chains cover every lane layout of the kernel: 16 pixels per lane (1, 2, ...,
64; 4, 8, ..., 64; 4), 9 (1, 3, 6, 12, 24, 48; 1, 3, 9, 27; 3), 4 (2, 6, 12,
whose finest square holds 4 pixels) and 1 (1, 2, 6, 12; 1, 5, 10); cross-lane
groups by butterflies (4, 16, 64 lanes) and by the LDS tree (9, 25, 36, 81,
100, 144, 256 lanes); one-level chains; ragged images and shifted lattices on
each axis.
"""
import numpy as np
import pytest

import oracle
import smre_inputs as gi
from nested_kkt import phase_squares

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CHAINS = {
    "p2_64": [1, 2, 4, 8, 16, 32, 64],
    "r3_48": [1, 3, 6, 12, 24, 48],
    "r3_27": [1, 3, 9, 27],
    "m2_12": [1, 2, 6, 12],
    "f2_12": [2, 6, 12],
    "p1_10": [1, 5, 10],
    "f4_64": [4, 8, 16, 32, 64],
    "one_3": [3],
    "one_4": [4],
}


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


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=dtype)


def phases_for(sides):
    """The lattice at rest, shifted on both axes, on one axis only, and with a
    raised lowest level."""
    B = sides[-1]
    n = len(sides)
    return [(0, 0, 0), (B // 2, B // 2, 0), (0, max(1, B // 3) % B, min(1, n - 1)),
            (max(1, B // 4) % B, 0, n // 2)]


def image(H, W, seed):
    # emitters on noise above the per-pixel bound: coarse squares bind too
    return gi.emitters(H, W, n_e=max(3, H * W // 400), seed=seed) + \
        1.3 * gi.gaussian(H, W, seed=seed + 1)


@pytest.mark.parametrize("name", list(CHAINS))
@pytest.mark.parametrize("H,W", [(70, 75), (100, 61)])
def test_fp64_matches_oracle(ctx, name, H, W):
    sides = CHAINS[name]
    r2 = oracle.chi2_bounds(sides)
    ph = phases_for(sides)
    x0 = image(H, W, H + len(sides))
    ref, n_ref = oracle.icd_nested(x0, sides, r2, ph, tol=1e-13, max_inner=100000)
    x = dev(x0)
    rep = ctx.incomplete_nested(x, sides, r2, ph, tol=1e-13, mode=0, max_inner=100000)
    err = relerr(x.cpu().numpy(), ref)
    print(f"{name} {H}x{W}: {err:.2e}, inner {rep['inner_sweeps']} (oracle {n_ref})")
    assert rep["converged"] == 1
    assert err <= 1e-10


@pytest.mark.parametrize("name", ["p2_64", "r3_48", "m2_12"])
def test_fp32_matches_oracle(ctx, name):
    sides = CHAINS[name]
    r2 = oracle.chi2_bounds(sides)
    ph = phases_for(sides)
    x0 = image(128, 97, 5).astype(np.float32).astype(np.float64)
    ref, _ = oracle.icd_nested(x0, sides, r2, ph, tol=1e-13, max_inner=100000)
    x = dev(x0, torch.float32)
    ctx.incomplete_nested(x, sides, r2, ph, tol=1e-7, mode=0, max_inner=100000)
    err = relerr(x.double().cpu().numpy(), ref)
    print(f"FP32 {name}: {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("name", ["r3_48", "p2_64"])
def test_one_inner_sweep_exact_and_counted(ctx, name):
    """max_inner = 1: one Dykstra sweep per block (no stopping decision), so the
    result matches the oracle to rounding, every block is reported capped, and
    the counters equal the squares (and their pixels) of the phases."""
    sides = CHAINS[name]
    r2 = oracle.chi2_bounds(sides)
    ph = phases_for(sides)
    H, W = 90, 77
    x0 = image(H, W, 9)
    ref, _ = oracle.icd_nested(x0, sides, r2, ph, tol=1e-13, max_inner=1)
    x = dev(x0)
    rep = ctx.incomplete_nested(x, sides, r2, ph, tol=1e-13, mode=0, max_inner=1)
    assert relerr(x.cpu().numpy(), ref) <= 1e-12
    assert rep["converged"] == 0
    nsq = npx = 0
    for sy, sx, lo in ph:
        sq = phase_squares(H, W, sides, sy, sx, lo)
        for j in sq:
            nsq += len(sq[j])
            npx += len(sq[j]) * sides[j] ** 2
    B = sides[-1]
    nblk = sum(((H - (sy - B if sy else 0) + B - 1) // B) * ((W - (sx - B if sx else 0) + B - 1) // B)
               for sy, sx, _ in ph)
    assert rep["window_projections"] == nsq
    assert rep["pixel_updates"] == npx
    assert rep["inner_sweeps"] == nblk


def test_paper_rule_close_to_oracle(ctx):
    sides = CHAINS["r3_48"]
    r2 = oracle.chi2_bounds(sides)
    ph = phases_for(sides)
    x0 = image(160, 150, 12)
    ref, n_ref = oracle.icd_nested(x0, sides, r2, ph, tol=1e-3, mode=oracle.TOL_MEANABS,
                                   max_inner=10000)
    x = dev(x0)
    rep = ctx.incomplete_nested(x, sides, r2, ph, tol=1e-3, mode=1, max_inner=10000)
    # same stopping rule; a decision may flip only on rounding-level ties
    assert relerr(x.cpu().numpy(), ref) <= 1e-3
    assert rep["inner_sweeps"] == pytest.approx(n_ref, rel=0.01)


@pytest.mark.parametrize("dtype,gate", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_k6_paper_icd(ctx, dtype, gate):
    """smre_dykstra_incomplete with K = 6 (64 x 64 blocks) against the paper's
    ICD in the oracle, and bitwise equal to the nested call with the chain
    1, 2, ..., 64."""
    K = 6
    sides = [1 << k for k in range(K + 1)]
    r2 = oracle.chi2_bounds(sides)
    x0 = image(150, 139, 21).astype(np.float32).astype(np.float64)
    ref, _ = oracle.icd(x0, K, r2, tol=1e-13, mode=oracle.TOL_MAXABS, max_inner=100000)
    tol = 1e-13 if dtype == torch.float64 else 1e-7
    a = dev(x0, dtype)
    rep = ctx.incomplete(a, K, r2, tol=tol, mode=0, max_inner=100000)
    b = dev(x0, dtype)
    ctx.incomplete_nested(b, sides, r2, oracle.icd_paper_phases(K), tol=tol, mode=0,
                          max_inner=100000)
    assert torch.equal(a, b)
    assert rep["region"] == 64
    assert relerr(a.double().cpu().numpy(), ref) <= gate


def test_k5_chain_matches_wave_kernel(ctx):
    """The chain 1, ..., 32 on the nested kernel against the one-wave-per-block
    kernel of smre_dykstra_incomplete (K = 5): two layouts, one method."""
    K = 5
    sides = [1 << k for k in range(K + 1)]
    r2 = oracle.chi2_bounds(sides)
    x0 = image(120, 101, 4)
    a = dev(x0)
    ctx.incomplete(a, K, r2, tol=1e-13, mode=0, max_inner=100000)
    b = dev(x0)
    ctx.incomplete_nested(b, sides, r2, oracle.icd_paper_phases(K), tol=1e-13, mode=0,
                          max_inner=100000)
    assert relerr(b.cpu().numpy(), a.cpu().numpy()) <= 1e-11


def test_frames_equal_single_calls(ctx):
    sides = CHAINS["r3_48"]
    r2 = oracle.chi2_bounds(sides)
    ph = phases_for(sides)
    frames = np.stack([image(64, 70, 30 + f) for f in range(3)])
    xs = dev(frames, torch.float32)
    rep = ctx.incomplete_nested(xs, sides, r2, ph, tol=1e-3, mode=1, max_inner=10000)
    for f in range(3):
        one = dev(frames[f], torch.float32)
        ctx.incomplete_nested(one, sides, r2, ph, tol=1e-3, mode=1, max_inner=10000)
        assert torch.equal(one, xs[f])
    assert rep["inner_sweeps"] > 0


def test_reported_violation_is_the_full_family(ctx):
    """max_violation: the largest window sum over every position of each
    level's side, relative to its bound (brute force with cumulative sums)."""
    sides = CHAINS["m2_12"]
    r2 = oracle.chi2_bounds(sides)
    ph = phases_for(sides)
    x0 = image(80, 90, 40)
    x = dev(x0)
    rep = ctx.incomplete_nested(x, sides, r2, ph, tol=1e-3, mode=1, max_inner=10000)
    z = x.cpu().numpy()
    c = np.zeros((81, 91))
    c[1:, 1:] = np.cumsum(np.cumsum(z * z, 0), 1)
    worst = -np.inf
    for s, r in zip(sides, r2):
        win = c[s:, s:] - c[:-s, s:] - c[s:, :-s] + c[:-s, :-s]
        worst = max(worst, float(np.max(win)) / r - 1)
    assert rep["max_violation"] == pytest.approx(worst, abs=1e-9)


@pytest.mark.parametrize("sides,phases", [
    ([2, 3], [(0, 0, 0)]),               # 2 does not divide 3
    ([1, 5, 10, 20, 40], [(0, 0, 0)]),   # no level fits the lanes (1600 needed)
    ([1, 3, 6], [(6, 0, 0)]),            # shift >= block side
    ([1, 3, 6], [(0, 0, 3)]),            # no level 3
    ([1, 2, 4, 8, 16, 32, 64, 128], [(0, 0, 0)]),
])
def test_rejects_bad_arguments(ctx, smre, sides, phases):
    x = dev(np.zeros((200, 200)))
    with pytest.raises(smre.SmreError) as e:
        ctx.incomplete_nested(x, sides, [1.0] * len(sides), phases)
    assert e.value.code == -1
