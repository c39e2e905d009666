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
