"""GPU serving: continuous batching of projection requests.

A request's result does not depend on what else is on the device: the server
runs the batched kernels with region side 16, so each request gets exactly the
arithmetic of a single-image solve with R = 16 -- same bits, same stopping
sweep -- whether it runs alone or joins a running mix.
"""
import time

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


def wait(srv, ticket, shape, timeout=120.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        r = srv.poll(ticket, shape)
        if r is not None:
            return r
        time.sleep(0.002)
    raise TimeoutError(ticket)


def single(smre, x0, sides, r2, tol, max_sweeps):
    ctx = smre.Context(0)
    x = torch.from_numpy(x0).cuda()
    rc, rep = ctx.project(x, sides, r2, tol=tol, max_sweeps=max_sweeps, region=16)
    ctx.close()
    return x.cpu().numpy(), rep


def test_alone_and_in_mix_identical(smre):
    reqs = []
    for k, (H, W) in enumerate([(64, 64), (96, 80), (48, 130), (128, 128), (70, 70)]):
        x0 = gi.emitters(H, W, n_e=max(2, H * W // 300), seed=k).astype(np.float32)
        sides = list(range(1, 9)) if k % 2 == 0 else [1, 2, 3, 5, 7]
        reqs.append((x0, sides, oracle.chi2_bounds(sides), [1e-4, 1e-5][k % 2]))
    srv = smre.Server(max_active=3, queue_cap=64)
    # staggered arrivals: later requests join while earlier ones are running
    tickets = [srv.submit(*reqs[0][:3], tol=reqs[0][3], max_sweeps=4000)]
    t0 = time.time()
    while srv.stats()["active"] < 1 and time.time() - t0 < 30:
        time.sleep(0.001)
    for x0, sides, r2, tol in reqs[1:]:
        tickets.append(srv.submit(x0, sides, r2, tol=tol, max_sweeps=4000))
        time.sleep(0.003)
    outs = [wait(srv, t, r[0].shape) for t, r in zip(tickets, reqs)]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs)
    # the mix really shared the device: several requests at once, and requests
    # admitted while others were part-way through their sweeps
    print(f"peak active {st['peak_active']}, joined a running mix {st['joined_running']}")
    assert st["peak_active"] >= 2 and st["joined_running"] >= 1
    for (x0, sides, r2, tol), (rc, z, rep, lat) in zip(reqs, outs):
        ref, rep1 = single(smre, x0, sides, r2, tol, 4000)
        assert rc == 0 and rep["converged"] == 1
        assert rep["sweeps"] == rep1["sweeps"]
        assert np.array_equal(z, ref)
        assert lat > 0


def test_bf16_increments_alone_and_served_identical(smre):
    """A server storing increments in BF16 gives each request the bits of the
    same image solved alone with BF16 increments at R = 16."""
    reqs = []
    for k, (H, W) in enumerate([(64, 72), (90, 64), (50, 100)]):
        x0 = gi.emitters(H, W, n_e=max(2, H * W // 300), seed=20 + k).astype(np.float32)
        sides = list(range(1, 9)) if k != 1 else [1, 2, 4, 12]
        reqs.append((x0, sides, oracle.chi2_bounds(sides)))
    srv = smre.Server(max_active=3, inc=smre.INC_BF16)
    tickets = [srv.submit(x0, s, r2, tol=1e-5, max_sweeps=3000) for x0, s, r2 in reqs]
    outs = [wait(srv, t, r[0].shape) for t, r in zip(tickets, reqs)]
    srv.close()
    ctx = smre.Context(0)
    for (x0, sides, r2), (rc, z, rep, lat) in zip(reqs, outs):
        x = torch.from_numpy(x0).cuda()
        _, rep1 = ctx.project(x, sides, r2, tol=1e-5, max_sweeps=3000, region=16,
                              inc=smre.INC_BF16)
        assert rep["sweeps"] == rep1["sweeps"]
        assert np.array_equal(z, x.cpu().numpy())
    ctx.close()


def test_matches_oracle_per_sweep(smre):
    x0 = gi.emitters(80, 72, n_e=20, seed=3).astype(np.float32)
    sides = list(range(1, 9))
    r2 = oracle.chi2_bounds(sides)
    srv = smre.Server(max_active=2)
    t = srv.submit(x0, sides, r2, tol=0, max_sweeps=3)
    rc, z, rep, lat = wait(srv, t, x0.shape)
    srv.close()
    ref, _, _ = oracle.dykstra(x0.astype(np.float64), sides, r2, tol=0, max_sweeps=3,
                               order=oracle.ORDER_REGION, region=16)
    assert rep["sweeps"] == 3
    assert np.max(np.abs(z - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_admission_by_footprint_and_errors(smre):
    x0 = gi.emitters(256, 256, n_e=50, seed=4).astype(np.float32)
    sides = list(range(1, 9))
    r2 = oracle.chi2_bounds(sides)
    # arena for about one 256^2 request (its increments are ~54 MB)
    srv = smre.Server(hbm_budget_bytes=80 << 20, max_active=4, queue_cap=2)
    with pytest.raises(smre.SmreError) as e:
        srv.submit(gi.emitters(1024, 1024, n_e=10, seed=1).astype(np.float32), sides, r2)
    assert e.value.code == -4  # can never fit
    bad = x0.copy()
    bad[3, 3] = np.nan
    with pytest.raises(smre.SmreError) as e:
        srv.submit(bad, sides, r2)
    assert e.value.code == -2
    t1 = srv.submit(x0, sides, r2, tol=1e-4, max_sweeps=300)
    t0 = time.time()
    while srv.stats()["active"] < 1 and time.time() - t0 < 30:
        time.sleep(0.001)
    t2 = srv.submit(x0, sides, r2, tol=1e-4, max_sweeps=300)
    t3 = srv.submit(x0, sides, r2, tol=1e-4, max_sweeps=300)
    with pytest.raises(smre.SmreError) as e:
        srv.submit(x0, sides, r2, tol=1e-4, max_sweeps=300)
    assert e.value.code == -5  # queue full while the arena holds one request at a time
    res = [wait(srv, t, x0.shape) for t in (t1, t2, t3)]
    assert all(r[0] in (0, 1) for r in res)
    assert np.array_equal(res[0][1], res[1][1])
    assert srv.poll(t1, x0.shape)[0] == -8  # released
    st = srv.stats()
    assert st["completed"] == 3 and st["rejected"] >= 2
    srv.close()
