"""GPU serving: requests of two geometries arriving over time are served by the
continuous-batching loop; every result is bit-identical to solving that
request alone, and the C1-geometry results match the FP64 oracle's
reconstruction with the same iteration counts (relative L2 1e-4)."""
import numpy as np
import pytest

import synth
from synth.configs import Geometry

pytestmark = pytest.mark.gpu


def test_served_results_equal_solo_solves(orc, record):
    import torch
    from paper_1310_1434_amd import air
    from paper_1310_1434_amd.serve import GpuExecutor, Request, Server, latency_stats

    lam, mu, n_cg = 0.005, 1.0, 4
    g1 = synth.workload("c1").geom
    g2 = Geometry("fan", n=96, pixel=1.5, n_views=90, n_bins=140, bin=1.6, sod=500.0, sdd=900.0)
    w1 = synth.workload("c1")
    reqs = []
    for i in range(7):
        g = g1 if i % 3 else g2
        if g is g1:
            y = synth.make_case(w1, i)["y"]
        else:
            y = np.random.default_rng(i).uniform(0.0, 3.0, (g.n_views, g.n_bins))
        reqs.append(Request(i, g, y.astype(np.float32), n_outer=3 + i % 3, arrival=0.004 * i))
    ex = GpuExecutor(lam, mu, n_cg, max_outer=6, capacity=2)
    srv = Server(ex, hbm_budget=1 << 34, capacity=2)
    done = srv.run(reqs)
    assert all(r.error is None for r in done)
    st = latency_stats(done)
    assert st["count"] == 7
    admitted_during = sum(1 for r in done for o in done if o.rid != r.rid and o.admitted is not None
                          and r.admitted < o.finished and r.admitted > o.admitted)
    assert admitted_during > 0                       # some request joined while another ran
    for r in done:
        plan = air.Plan(r.geom)
        x, res = plan.solve(torch.from_numpy(r.y[None]).cuda(), lam, mu, r.n_outer, n_cg)
        torch.cuda.synchronize()
        assert np.array_equal(x[0].cpu().numpy(), r.x), r.rid
        assert np.array_equal(res[0].cpu().numpy(), r.resid), r.rid
        if r.geom is g1:
            xr, rr = orc.solve(orc.Geom(g1), r.y.astype(np.float64), lam, mu, r.n_outer, n_cg)
            e = float(np.linalg.norm(r.x.astype(np.float64) - xr) / np.linalg.norm(xr))
            record(f"rel_l2_served_c1_req{r.rid}", e)
            assert e < 1e-4, (r.rid, e)
            np.testing.assert_allclose(r.resid, rr, rtol=1e-3)
