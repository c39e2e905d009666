"""air_solve_noalloc (the allocation-free solve, for callers that cannot
allocate device memory) against air_solve through the C ABI: two calls in a
row on the library's static scratch, the second with a smaller input, each
bit-identical to air_solve with a caller workspace; batches beyond the static
scratch are refused before any GPU work."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1310_1434_amd import air
    return torch, air


def _solve_ws(torch, plan, ys, x0, n_outer, n_cg):
    x, r = plan.solve(torch.from_numpy(ys).cuda(), 0.005, 1.0, n_outer, n_cg, x0=torch.from_numpy(x0).cuda())
    torch.cuda.synchronize()
    return x.cpu().numpy(), r.cpu().numpy()


def _solve_noalloc(torch, plan, ys, x0, n_outer, n_cg):
    y = torch.from_numpy(ys).cuda()
    x = torch.from_numpy(x0).cuda()
    r = torch.full((ys.shape[0], n_outer), -1.0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    print(f"air_solve_noalloc: batch {ys.shape[0]}, {plan.n}^2 x {plan.n_views} views", flush=True)
    plan.solve_noalloc(y, x, 0.005, 1.0, n_outer, n_cg, resid=r)
    torch.cuda.synchronize()
    return x.cpu().numpy(), r.cpu().numpy()


def test_noalloc_matches_workspace_solve_twice(env):
    """C1 geometry: a batch of 9 (air_solve splits it over two streams, the
    allocation-free call keeps one: same bits), then a batch of 2 with a start
    image, on the same static scratch."""
    torch, air = env
    w = synth.workload("c1")
    ys = np.stack([synth.make_case(w, s)["y"] for s in range(9)]).astype(np.float32)
    x0 = np.zeros((9, w.geom.n, w.geom.n), np.float32)
    plan = air.Plan(w.geom)
    xa, ra = _solve_noalloc(torch, plan, ys, x0, 3, 4)
    xb, rb = _solve_ws(torch, plan, ys, x0, 3, 4)
    assert np.array_equal(xa, xb) and np.array_equal(ra, rb)
    x0s = np.random.default_rng(4).uniform(0, 0.02, (2, w.geom.n, w.geom.n)).astype(np.float32)
    xa2, ra2 = _solve_noalloc(torch, plan, ys[5:7].copy(), x0s, 2, 3)
    xb2, rb2 = _solve_ws(torch, plan, ys[5:7].copy(), x0s, 2, 3)
    assert np.array_equal(xa2, xb2) and np.array_equal(ra2, rb2)
    assert np.isfinite(xa2).all() and np.abs(xa2 - xa[5:7]).max() > 0      # a different solve, not stale data


def test_noalloc_size_limit_c2(env):
    """512^2, 720 views x 736 bins: 9 images fit the static scratch (and give
    air_solve's bits), 10 are refused with AIR_E_NOMEM before any work."""
    torch, air = env
    w = synth.workload("c2")
    plan = air.Plan(w.geom)
    y = synth.make_case(w, 0)["y"].astype(np.float32)
    ys = np.stack([y] * 9)
    x0 = np.zeros((9, w.geom.n, w.geom.n), np.float32)
    xa, ra = _solve_noalloc(torch, plan, ys, x0, 1, 1)
    xb, rb = _solve_ws(torch, plan, ys, x0, 1, 1)
    assert np.array_equal(xa, xb) and np.array_equal(ra, rb)
    y10 = torch.zeros((10, w.geom.n_views, w.geom.n_bins), device="cuda")
    x10 = torch.zeros((10, w.geom.n, w.geom.n), device="cuda")
    with pytest.raises(air.AirError) as e:
        plan.solve_noalloc(y10, x10, 0.005, 1.0, 1, 1)
    assert e.value.status == air.AIR_E_NOMEM
    assert "static" in str(e.value)
    assert torch.count_nonzero(x10).item() == 0
