"""Every ICD entry point on a non-finite input: SMRE_ENONFINITE and the image
left exactly as it came (the input check is read by the phase kernels, not by
the host before them), and the next call on a clean image unaffected by the
raised flag (bitwise equal to the same call in a fresh state)."""
import numpy as np
import pytest

import oracle
import smre_inputs as gi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K = 3
R2 = oracle.chi2_bounds([1 << k for k in range(K + 1)])
CHAIN = [1, 3, 6, 12]
CR2 = oracle.chi2_bounds(CHAIN)
CPH = [(0, 0, 0), (6, 6, 1)]


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


CALLS = {
    "incomplete": lambda c, x: c.incomplete(x, K, R2, tol=1e-6, mode=0),
    "noalloc": lambda c, x: c.incomplete_noalloc(x, K, R2, tol=1e-6, mode=0),
    "frames": lambda c, x: c.incomplete_frames(x, K, R2, tol=1e-6, mode=0),
    "family": lambda c, x: c.incomplete_family(x, K, R2, [(0, 0, 0), (1, 2, 0), (4, 0, 1)],
                                               tol=1e-6, mode=0),
    "nested": lambda c, x: c.incomplete_nested(x, CHAIN, CR2, CPH, tol=1e-6, mode=0),
    "k6": lambda c, x: c.incomplete(x, 6, oracle.chi2_bounds([1 << k for k in range(7)]),
                                    tol=1e-6, mode=0),
}


def image(name, seed):
    if name == "frames":
        return np.stack([3.0 * gi.gaussian(50, 61, seed=seed + f) for f in range(3)])
    return 3.0 * gi.gaussian(70, 83, seed=seed)


@pytest.mark.parametrize("name", list(CALLS))
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_nonfinite_leaves_image_and_next_call(ctx, smre, name, bad, dtype):
    run = CALLS[name]
    x0 = image(name, 7)
    x = torch.from_numpy(x0).to("cuda", dtype=dtype)
    # the far corner of the last frame: every phase touches the rest
    if x.dim() == 3:
        x[-1, -1, -1] = bad
    else:
        x[-1, -1] = bad
    before = x.clone()
    with pytest.raises(smre.SmreError) as e:
        run(ctx, x)
    assert e.value.code == -2
    torch.cuda.synchronize()
    same = (x == before) | (torch.isnan(x) & torch.isnan(before))
    assert bool(same.all())

    # a clean image after the failure: equal to the same call in a new context
    clean = image(name, 11)
    a = torch.from_numpy(clean).to("cuda", dtype=dtype)
    ra = run(ctx, a)
    fresh = smre.Context(0)
    try:
        b = torch.from_numpy(clean).to("cuda", dtype=dtype)
        rb = run(fresh, b)
    finally:
        fresh.close()
    assert torch.equal(a, b)
    assert not torch.equal(a, torch.from_numpy(clean).to("cuda", dtype=dtype))
    for k in ("inner_sweeps", "window_projections", "pixel_updates", "converged"):
        assert ra[k] == rb[k], k
    assert ra["max_violation"] == rb["max_violation"]
