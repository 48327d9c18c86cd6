"""GPU parity of the incomplete Dykstra over the frames of a movie.

Every frame of smre_dykstra_incomplete_frames must be exactly what
smre_dykstra_incomplete gives for that frame alone (same kernel, same
arithmetic: compared bitwise) and match the ICD oracle run frame by frame
(FP64 1e-10, FP32 1e-5 relative to max|z|, converged inner loops).  Shapes
with ragged block edges, strided rows, K = 0..5, fewer phases than K + 1; the
reported counts are the sums of the single-frame reports.  Full size: 3091
frames of 512 x 512 in one call (the bench's launch configuration), sampled
frames against single-frame calls and the oracle.
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


def bounds(K):
    return oracle.chi2_bounds([1 << k for k in range(K + 1)])


@pytest.mark.parametrize("n,H,W,K,phases", [(5, 70, 45, 3, None), (3, 37, 53, 2, None),
                                            (4, 40, 40, 0, None), (2, 96, 130, 5, None),
                                            (3, 64, 64, 4, 2)])
def test_frames_fp64_match_oracle_and_single(ctx, n, H, W, K, phases):
    print(f"frames fp64 n={n} {H}x{W} K={K} phases={phases}", flush=True)
    movie = gi.blinking_movie(n, H, W, n_e=max(3, H * W // 400), seed=K + n, dtype=np.float64)
    r2 = bounds(K)
    nph = K + 1 if phases is None else phases
    x = torch.from_numpy(movie).cuda()
    rep = ctx.incomplete_frames(x, K, r2, tol=1e-13, mode=0, max_inner=100000, num_phases=nph)
    got = x.cpu().numpy()
    inner = wp = pu = 0
    viol = -np.inf
    for f in range(n):
        ref, _ = oracle.icd(movie[f], K, r2, tol=1e-13, mode=oracle.TOL_MAXABS, max_inner=100000,
                            num_phases=nph)
        assert relerr(got[f], ref) <= 1e-10
        one = torch.from_numpy(movie[f].copy()).cuda()
        r1 = ctx.incomplete(one, K, r2, tol=1e-13, mode=0, max_inner=100000, num_phases=nph)
        assert np.array_equal(one.cpu().numpy(), got[f])
        inner += r1["inner_sweeps"]
        wp += r1["window_projections"]
        pu += r1["pixel_updates"]
        viol = max(viol, r1["max_violation"])
    assert rep["inner_sweeps"] == inner
    assert rep["window_projections"] == wp
    assert rep["pixel_updates"] == pu
    assert rep["max_violation"] == viol
    # the report's feasibility over the full family of the levels' sides
    fam = [1 << k for k in range(K + 1) if (1 << k) <= min(H, W)]
    fr2 = [r2[k] for k in range(K + 1) if (1 << k) <= min(H, W)]
    want = max(oracle.max_violation(got[f], fam, fr2) for f in range(n))
    assert viol == pytest.approx(want, rel=1e-12, abs=1e-13)


def test_frames_fp32_paper_rule_strided(ctx):
    # FP32 frames with a row stride larger than the width, the paper's
    # mean-abs rule; padding columns stay untouched
    n, H, W, K = 4, 64, 50, 4
    movie = gi.blinking_movie(n, H, W, n_e=12, seed=5)
    buf = torch.full((n, H, 64), 7.0, dtype=torch.float32, device="cuda")
    buf[:, :, :W] = torch.from_numpy(movie).cuda()
    x = buf[:, :, :W]
    r2 = bounds(K)
    ctx.incomplete_frames(x, K, r2, tol=1e-3, mode=1, max_inner=10000)
    got = buf.cpu().numpy()
    assert np.all(got[:, :, W:] == 7.0)
    for f in range(n):
        one = torch.from_numpy(movie[f].copy()).cuda()
        ctx.incomplete(one, K, r2, tol=1e-3, mode=1, max_inner=10000)
        assert np.array_equal(one.cpu().numpy(), got[f, :, :W])


def test_frames_fp32_converged_match_oracle(ctx):
    n, H, W, K = 3, 48, 80, 4
    movie = gi.blinking_movie(n, H, W, n_e=8, seed=9)
    r2 = bounds(K)
    x = torch.from_numpy(movie).cuda()
    ctx.incomplete_frames(x, K, r2, tol=1e-7, mode=0, max_inner=100000)
    got = x.double().cpu().numpy()
    for f in range(n):
        ref, _ = oracle.icd(movie[f].astype(np.float64), K, r2, tol=1e-13,
                            mode=oracle.TOL_MAXABS, max_inner=100000)
        assert relerr(got[f], ref) <= 1e-5


def test_frames_full_size_sampled(ctx):
    # 3091 frames of 512 x 512 in one call, as timed by the frames benchmark
    # (64 distinct generated frames, repeated)
    n, H, W, K = 3091, 512, 512, 4
    base = gi.blinking_movie(64, H, W, seed=0)
    src = torch.from_numpy(base).cuda()
    x = src[torch.arange(n, device="cuda") % 64].contiguous()
    r2 = bounds(K)
    rep = ctx.incomplete_frames(x, K, r2, tol=1e-3, mode=1, max_inner=10000)
    torch.cuda.synchronize()
    for f in (0, 1545, 3090):
        print(f"full-size frame {f}", flush=True)
        one = src[f % 64].clone()
        ctx.incomplete(one, K, r2, tol=1e-3, mode=1, max_inner=10000)
        assert torch.equal(one, x[f])
        assert torch.equal(x[f], x[f % 64])
    ref, _ = oracle.icd(base[1545 % 64].astype(np.float64), K, r2, tol=1e-3,
                        mode=oracle.TOL_MEANABS, max_inner=10000)
    # same stopping rule; a block's decision may flip on rounding-level ties
    assert relerr(x[1545].double().cpu().numpy(), ref) <= 1e-3
    assert rep["inner_sweeps"] > 0 and rep["max_violation"] < 1.0


def test_frames_reject_bad_arguments(ctx, smre):
    x = torch.zeros((2, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(smre.SmreError):  # K = 7: blocks of 128 exceed every kernel
        ctx.incomplete_frames(x, 7, np.ones(8))
    x[1, 3, 3] = float("nan")
    with pytest.raises(smre.SmreError):
        ctx.incomplete_frames(x, 2, bounds(2))


def test_frames_k6_equal_single_calls(ctx):
    """K = 6 frames run on the nested-hierarchy kernel: each frame bitwise
    equal to the same image projected alone."""
    K = 6
    r2 = bounds(K)
    frames = np.stack([gi.emitters(70, 81, n_e=6, seed=50 + f) for f in range(3)])
    xs = torch.from_numpy(frames).to("cuda", dtype=torch.float32)
    ctx.incomplete_frames(xs, K, r2, tol=1e-3, mode=1, max_inner=10000)
    for f in range(3):
        one = torch.from_numpy(frames[f]).to("cuda", dtype=torch.float32)
        ctx.incomplete(one, K, r2, tol=1e-3, mode=1, max_inner=10000)
        assert torch.equal(one, xs[f])


# ---------------------------------------------------------------- phase families

@pytest.mark.parametrize("H,W,K,phases", [
    (70, 45, 3, [(1, 0, 0), (0, 1, 0), (2, 0, 1), (0, 2, 1), (4, 4, 2)]),
    (37, 53, 2, [(0, 0, 0), (1, 0, 1), (0, 3, 1), (2, 1, 0)]),
    (64, 64, 4, [(1, 1, 0), (2, 0, 1), (0, 2, 1), (8, 8, 3), (0, 0, 4)]),
    (33, 96, 5, [(16, 0, 2), (0, 16, 3), (5, 7, 0)]),
])
def test_family_fp64_matches_oracle(ctx, H, W, K, phases):
    print(f"family fp64 {H}x{W} K={K} {phases}", flush=True)
    x0 = gi.emitters(H, W, n_e=max(3, H * W // 400), seed=K + H)
    r2 = bounds(K)
    ref, n_ref = oracle.icd_family(x0, K, r2, phases, tol=1e-13, max_inner=100000)
    x = torch.from_numpy(x0.copy()).cuda()
    rep = ctx.incomplete_family(x, K, r2, phases, tol=1e-13, mode=0, max_inner=100000)
    assert relerr(x.cpu().numpy(), ref) <= 1e-10
    assert rep["inner_sweeps"] == n_ref


def test_family_paper_phases_equal_incomplete(ctx):
    # the paper's family through the family entry point = the ICD call, bitwise
    n, H, W, K = 3, 64, 80, 4
    movie = gi.blinking_movie(n, H, W, n_e=10, seed=2)
    r2 = bounds(K)
    a = torch.from_numpy(movie).cuda()
    b = a.clone()
    ra = ctx.incomplete_frames(a, K, r2, tol=1e-3, mode=1)
    rb = ctx.incomplete_family(b, K, r2, oracle.icd_paper_phases(K), tol=1e-3, mode=1)
    assert torch.equal(a, b)
    assert ra["inner_sweeps"] == rb["inner_sweeps"]


def test_family_rejects_bad_phases(ctx, smre):
    x = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(smre.SmreError):
        ctx.incomplete_family(x, 2, bounds(2), [(4, 0, 0)])
    with pytest.raises(smre.SmreError):
        ctx.incomplete_family(x, 2, bounds(2), [(0, 0, 3)])
    with pytest.raises(smre.SmreError):
        ctx.incomplete_family(x, 2, bounds(2), [])


def test_frames_without_report_same_result(ctx, smre):
    # through the C ABI with report = NULL (the feasibility pass is skipped):
    # the frames come out bitwise as with a report
    import ctypes
    n, H, W, K = 3, 48, 64, 4
    movie = gi.blinking_movie(n, H, W, n_e=8, seed=12)
    r2 = np.ascontiguousarray(bounds(K))
    a = torch.from_numpy(movie).cuda()
    b = a.clone()
    ctx.incomplete_frames(a, K, r2, tol=1e-3, mode=1)
    rc = smre.lib().smre_dykstra_incomplete_frames(
        ctx._h, smre.F32, ctypes.c_void_p(b.data_ptr()), H, W, W, n, K,
        r2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1e-3, 1, 10000, K + 1,
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), None)
    torch.cuda.synchronize()
    assert rc == 0
    assert torch.equal(a, b)
