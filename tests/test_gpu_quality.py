"""GPU checks of the FBP / IR / AIR comparison: each arm against the FP64
oracle's arm on a small quality case, and the image-quality measures taken on
the GPU images against the same measures on the oracle images."""
import math

import numpy as np
import pytest

from paper_1310_1434_amd import quality as Q
from synth import quality as SQ
from synth.configs import Geometry

pytestmark = pytest.mark.gpu

GEOM = Geometry("fan", n=96, pixel=1.0, n_views=120, n_bins=150, bin=1.1, sod=300.0, sdd=500.0)
LAM, MU, N_OUTER, N_CG = 0.005, 1.0, 6, 4


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def cases():
    res = SQ.resolution_phantom(lps=(2.0, 3.0), ring=24.0, disc=44.0, length=8.0)
    con = SQ.contrast_phantom(contrasts=(0.002, 0.004), radii=(6.0,), ring=24.0, disc=44.0)
    return [(ph, SQ.make_quality_case(ph, GEOM, 2e4, 5 + k)) for k, ph in enumerate((res, con))]


@pytest.fixture(scope="module")
def arms(cases):
    import torch
    from paper_1310_1434_amd import air
    plan = air.Plan(GEOM, max_batch=2)
    s = Q.top_eigenvalue(plan, 0) / Q.top_eigenvalue(plan, 1)
    y = torch.from_numpy(np.stack([c["y"] for _, c in cases]).astype(np.float32)).cuda()
    out = Q.run_arms(plan, y, LAM, MU, N_OUTER, N_CG, s)
    torch.cuda.synchronize()
    return s, {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}


def test_ir_scale_is_the_operator_ratio(arms, orc):
    """The power-iteration ratio matches the same iteration on the oracle's
    normal operators (same start vector, same step count)."""
    s, _ = arms
    g = orc.Geom(GEOM)
    top = []
    for filt in (0, 1):
        x = Q.power_start(GEOM.n, 0).astype(np.float64)
        for _ in range(30):
            y = orc.apply_normal(g, x, 0.0, filt)
            lam = np.linalg.norm(y) / np.linalg.norm(x)
            x = y / np.linalg.norm(y)
        top.append(lam)
    assert s == pytest.approx(top[0] / top[1], rel=1e-3)
    assert s > 10.0      # A^T A is far larger than A'^T A (about the identity)


def test_arms_match_oracle_and_measures_agree(arms, cases, orc, record):
    s, gpu = arms
    g = orc.Geom(GEOM)
    for b, (ph, c) in enumerate(cases):
        y = c["y"].astype(np.float32).astype(np.float64)
        ref = {"FBP": orc.filtered_backproject(g, y, 1),
               "AIR": orc.solve(g, y, LAM, MU, N_OUTER, N_CG, filter=1)[0],
               "IR": orc.solve(g, y, LAM * s, MU * s, N_OUTER, N_CG, filter=0)[0]}
        for arm, tol in (("FBP", 1e-5), ("AIR", 1e-4), ("IR", 1e-4)):
            e = rel(gpu[arm][b], ref[arm])
            record(f"rel_l2_{arm}_{ph.name}", e)
            assert e < tol, (arm, ph.name, e)
            if ph.bar_groups:
                for gr in ph.bar_groups:
                    mg, mr = Q.bar_fwhm(gpu[arm][b], gr, GEOM.pixel), Q.bar_fwhm(ref[arm], gr, GEOM.pixel)
                    assert mg["resolved"] == mr["resolved"]
                    if mr["resolved"]:
                        assert abs(mg["fwhm_mm"] - mr["fwhm_mm"]) < 1e-3, (arm, gr.lp_per_cm)
            else:
                for tg, tr in zip(Q.target_cnrs(gpu[arm][b], ph, GEOM.pixel), Q.target_cnrs(ref[arm], ph, GEOM.pixel)):
                    assert math.isclose(tg["cnr"], tr["cnr"], rel_tol=1e-3), (arm, tg, tr)


# ----------------------------------------------------------------------------- the paper-shaped scan

@pytest.fixture(scope="module")
def paper_scans():
    """The paper-shaped scan (Materials: 350 x 350 at 1 mm, 528 detector
    pixels, 800 views, and its 25% subset of 200 views) of the resolution
    phantom, with Poisson noise at I0 = 2e4."""
    ph = SQ.resolution_phantom()
    full = SQ.make_quality_case(ph, SQ.paper_geometry(1), 2e4, 21)
    return ph, {1: (SQ.paper_geometry(1), full["y"], full["x_true"]),
                4: (SQ.paper_geometry(4), full["y"][::4].copy(), full["x_true"])}


@pytest.mark.parametrize("step", [1, 4], ids=["800_views", "200_views"])
def test_paper_scan_operators_and_solve(paper_scans, orc, record, step):
    """A, A'^T = A^T C and a 5 x 5 split-Bregman solve on the paper-shaped scan
    against the FP64 oracle: 1e-5 per operator apply, 1e-4 on the image."""
    import torch
    from paper_1310_1434_amd import air
    _, scans = paper_scans
    g, y, x_true = scans[step]
    print(f"paper-shaped scan, {g.n_views} views", flush=True)
    G = orc.Geom(g)
    plan = air.Plan(g, max_batch=1)
    x32 = x_true.astype(np.float32)
    yp = plan.project(torch.from_numpy(x32[None]).cuda())[0].cpu().numpy().astype(np.float64)
    e_a = rel(yp, orc.project(G, x32.astype(np.float64)))
    y32 = y.astype(np.float32)
    Y = torch.from_numpy(y32[None]).cuda()
    xb = plan.filtered_backproject(Y, 1)[0].cpu().numpy().astype(np.float64)
    e_atc = rel(xb, orc.filtered_backproject(G, y32.astype(np.float64), 1))
    xs, _ = plan.solve(Y, LAM, MU, 5, 5, with_resid=False)
    xr, _ = orc.solve(G, y32.astype(np.float64), LAM, MU, 5, 5)
    e_x = rel(xs[0].cpu().numpy().astype(np.float64), xr)
    record(f"rel_l2_A_paper_{g.n_views}", e_a)
    record(f"rel_l2_AtC_paper_{g.n_views}", e_atc)
    record(f"rel_l2_final_paper_{g.n_views}_5x5", e_x)
    assert e_a < 1e-5 and e_atc < 1e-5, (e_a, e_atc)
    assert e_x < 1e-4, e_x
