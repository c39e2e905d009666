"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative L2 over the whole output, accumulated in float64):
  per operator apply, float32 path ........................ 1e-5
  final split-Bregman image, float32 path ................. 1e-4
  final image, mixed-precision ramp ....................... 1e-3
  index tables ............................................ bit-exact (host tests)
Both sides receive the same float32-rounded inputs.
"""
import os

import numpy as np
import pytest

import synth
from synth.configs import Geometry

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def air():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1310_1434_amd import air
    return air


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def dev(t, x):
    return t.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()


def host(x):
    return x.detach().cpu().numpy().astype(np.float64)


RAGGED = Geometry("fan", n=100, pixel=1.1, n_views=37, n_bins=150, bin=1.3, sod=400.0, sdd=700.0)
SMALL_PAR = Geometry("parallel", n=40, pixel=1.0, n_views=30, n_bins=61, bin=1.0)
# bins much finer than pixels: a 16x16 tile's detector window spans ~350 bins,
# so the backprojector stages every view in several passes (about 6)
FINE = Geometry("fan", n=48, pixel=1.0, n_views=23, n_bins=960, bin=0.17, sod=120.0, sdd=200.0)


def geom(name):
    return {"c1": synth.workload("c1").geom, "c2": synth.workload("c2").geom,
            "c2_25": synth.workload("c2_25").geom, "ragged": RAGGED, "small_par": SMALL_PAR,
            "fine": FINE}[name]


def image_for(name, seed=0):
    if name in ("c1", "c2", "c2_25"):
        w = synth.workload(name)
        return synth.make_case(w, seed)["x_true"]
    g = geom(name)
    return np.random.default_rng(seed).uniform(0, 0.03, (g.n, g.n))


def sino_for(name, seed=0):
    if name in ("c1", "c2", "c2_25"):
        return synth.make_case(synth.workload(name), seed)["y"]
    g = geom(name)
    return np.random.default_rng(seed + 100).uniform(0, 5, (g.n_views, g.n_bins))


# ----------------------------------------------------------------------------- operators

@pytest.mark.parametrize("name", ["c1", "ragged", "c2"])
def test_project_parity(air, torch_mod, orc, record, name):
    g = geom(name)
    x = image_for(name).astype(np.float32)
    plan = air.Plan(g, max_batch=1)
    y = host(plan.project(dev(torch_mod, x[None])))[0]
    ref = orc.project(orc.Geom(g), x.astype(np.float64))
    record("rel_l2_A", rel(y, ref))
    assert rel(y, ref) < 1e-5


@pytest.mark.parametrize("prec", ["fp32", "mixed_f16", "mixed_bf16"])
@pytest.mark.parametrize("name", ["c1", "ragged", "c2"])
def test_ramp_parity(air, torch_mod, orc, record, name, prec):
    g = geom(name)
    y = sino_for(name).astype(np.float32)
    plan = air.Plan(g, max_batch=1, precision=prec)
    yf = host(plan.ramp(dev(torch_mod, y[None])))[0]
    ref = orc.ramp(orc.Geom(g), y.astype(np.float64))
    record("rel_l2_C", rel(yf, ref))
    assert rel(yf, ref) < 1e-5, (name, prec, rel(yf, ref))


@pytest.mark.parametrize("prec", ["mixed_f16", "mixed_bf16"])
def test_split_ramp_column_tiles(air, torch_mod, orc, record, prec):
    """The 16-bit ramp kernels cover 32, 64 or 128 columns per block depending
    on the launch size (C2: batch 1, 8 and 16).  A column's sums do not depend
    on the tile width, so every image's output is the same bits in each, and
    it matches the oracle."""
    g = geom("c2")
    ys = np.stack([sino_for("c2", s % 3) * (1 + 0.1 * s) for s in range(16)]).astype(np.float32)
    plan = air.Plan(g, max_batch=16, precision=prec)
    y16 = host(plan.ramp(dev(torch_mod, ys)))
    y8 = host(plan.ramp(dev(torch_mod, ys[:8])))
    y1 = host(plan.ramp(dev(torch_mod, ys[5:6])))[0]
    assert np.array_equal(y16[:8], y8)
    assert np.array_equal(y16[5], y1)
    for b in (0, 15):
        e = rel(y16[b], orc.ramp(orc.Geom(g), ys[b].astype(np.float64)))
        record(f"rel_l2_C_{prec}_b16", e)
        assert e < 1e-5, (b, e)


@pytest.mark.parametrize("filt", [0, 1])
@pytest.mark.parametrize("name", ["c1", "ragged", "fine", "c2"])
def test_filtered_backproject_parity(air, torch_mod, orc, record, name, filt):
    g = geom(name)
    y = sino_for(name).astype(np.float32)
    plan = air.Plan(g, max_batch=1)
    x = host(plan.filtered_backproject(dev(torch_mod, y[None]), filter=filt))[0]
    ref = orc.filtered_backproject(orc.Geom(g), y.astype(np.float64), filt)
    record("rel_l2_AtC" if filt else "rel_l2_At", rel(x, ref))
    assert rel(x, ref) < 1e-5, rel(x, ref)


@pytest.mark.parametrize("name", ["c1", "ragged", "c2"])
def test_normal_operator_parity(air, torch_mod, orc, record, name):
    g = geom(name)
    x = image_for(name).astype(np.float32)
    plan = air.Plan(g, max_batch=1)
    out = host(plan.normal_apply(dev(torch_mod, x[None]), 1.0, 1))[0]
    ref = orc.apply_normal(orc.Geom(g), x.astype(np.float64), 1.0, 1)
    record("rel_l2_M", rel(out, ref))
    assert rel(out, ref) < 1e-5


@pytest.mark.parametrize("n", [37, 128])
def test_framelet_parity(air, torch_mod, orc, n):
    g = Geometry("parallel", n=n, pixel=1.0, n_views=4, n_bins=n + 5, bin=1.0)
    plan = air.Plan(g, max_batch=1)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((2, n, n)).astype(np.float32)
    z = host(plan.framelet(dev(torch_mod, x)))
    for b in range(2):
        assert rel(z[b], orc.framelet(x[b].astype(np.float64))) < 1e-6
    zz = rng.standard_normal((2, 9, n, n)).astype(np.float32)
    xa = host(plan.framelet_adjoint(dev(torch_mod, zz)))
    for b in range(2):
        assert rel(xa[b], orc.framelet_adjoint(zz[b].astype(np.float64))) < 1e-6


@pytest.mark.parametrize("g", [Geometry("fan", n=12, pixel=1.0, n_views=9, n_bins=21, bin=1.0, sod=40.0, sdd=70.0),
                               Geometry("fan", n=10, pixel=1.0, n_views=5, n_bins=150, bin=0.19, sod=40.0, sdd=70.0),
                               Geometry("parallel", n=19, pixel=0.8, n_views=7, n_bins=30, bin=1.1)],
                         ids=["fan", "fan_fine_bins", "parallel_ragged"])
def test_gpu_adjoint_is_exact_transpose(air, torch_mod, g):
    """Dense A from unit images and dense A^T from unit rays agree bit for bit:
    the gather backprojector evaluates exactly the forward projector's weights
    (also when a tile's window needs several staging passes, and on tiles cut
    by the image edge)."""
    n, nr = g.n, g.n_views * g.n_bins
    plan = air.Plan(g, max_batch=max(n * n, nr))
    t = torch_mod
    A = host(plan.project(t.eye(n * n, device="cuda").reshape(n * n, n, n))).reshape(n * n, nr).T
    At = host(plan.filtered_backproject(t.eye(nr, device="cuda").reshape(nr, g.n_views, g.n_bins), 0))
    At = At.reshape(nr, n * n).T
    assert np.array_equal(A.T, At)
    assert (A > 0).sum() > nr


@pytest.mark.parametrize("g", [Geometry("parallel", n=1, pixel=1.0, n_views=6, n_bins=5, bin=0.7),
                               Geometry("fan", n=2, pixel=1.0, n_views=7, n_bins=9, bin=0.6, sod=20.0, sdd=35.0),
                               Geometry("fan", n=3, pixel=0.9, n_views=8, n_bins=12, bin=0.5, sod=25.0, sdd=40.0),
                               Geometry("fan", n=17, pixel=1.0, n_views=9, n_bins=31, bin=1.0, sod=60.0, sdd=100.0),
                               Geometry("parallel", n=33, pixel=1.0, n_views=11, n_bins=50, bin=0.9)],
                         ids=["n1", "n2", "n3", "n17", "n33"])
def test_gpu_adjoint_is_exact_transpose_at_image_edges(air, torch_mod, g):
    """The same bit-for-bit transpose on images whose last tile starts on the
    last row or column (n = 17, 33) or that are smaller than a pixel pair
    (n = 1, 2, 3): the backprojector's window table covers the clamped
    stand-in pixels of pairs cut by the image edge."""
    n, nr = g.n, g.n_views * g.n_bins
    plan = air.Plan(g, max_batch=max(n * n, nr))
    t = torch_mod
    A = host(plan.project(t.eye(n * n, device="cuda").reshape(n * n, n, n))).reshape(n * n, nr).T
    At = host(plan.filtered_backproject(t.eye(nr, device="cuda").reshape(nr, g.n_views, g.n_bins), 0))
    At = At.reshape(nr, n * n).T
    assert np.array_equal(A.T, At)
    assert (A > 0).sum() >= n * n


def test_gpu_adjoint_dot_product_c2(air, torch_mod):
    g = geom("c2")
    plan = air.Plan(g, max_batch=1)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((1, g.n, g.n)).astype(np.float32)
    y = rng.standard_normal((1, g.n_views, g.n_bins)).astype(np.float32)
    ax = host(plan.project(dev(torch_mod, x)))
    aty = host(plan.filtered_backproject(dev(torch_mod, y), 0))
    lhs = float(np.sum(ax * y.astype(np.float64)))
    rhs = float(np.sum(x.astype(np.float64) * aty))
    assert abs(lhs - rhs) < 1e-5 * np.linalg.norm(ax) * np.linalg.norm(y)


def test_operator_batch_matches_single(air, torch_mod):
    g = geom("c1")
    plan = air.Plan(g, max_batch=3)
    xs = np.stack([image_for("c1", s) for s in range(3)]).astype(np.float32)
    yb = host(plan.project(dev(torch_mod, xs)))
    for b in range(3):
        y1 = host(plan.project(dev(torch_mod, xs[b:b + 1])))[0]
        assert np.array_equal(y1, yb[b])


@pytest.mark.parametrize("batch", [2, 3, 5, 9, 16, 33])
def test_backprojection_batch_matches_single(air, torch_mod, batch):
    """Every image gets the same bits whatever group of images it is processed
    in (groups of 2, 4, 8 or 16, with idle lanes in the last group)."""
    g = geom("ragged")
    plan = air.Plan(g, max_batch=batch)
    ys = np.stack([sino_for("ragged", s) for s in range(batch)]).astype(np.float32)
    for filt in (0, 1):
        xb = host(plan.filtered_backproject(dev(torch_mod, ys), filter=filt))
        for b in range(batch):
            x1 = host(plan.filtered_backproject(dev(torch_mod, ys[b:b + 1]), filter=filt))[0]
            assert np.array_equal(x1, xb[b]), (filt, b)
    xs = np.random.default_rng(batch).uniform(0, 0.03, (batch, g.n, g.n)).astype(np.float32)
    yb = host(plan.project(dev(torch_mod, xs)))
    for b in range(batch):
        assert np.array_equal(host(plan.project(dev(torch_mod, xs[b:b + 1])))[0], yb[b])


@pytest.mark.parametrize("g", [Geometry("parallel", n=45, pixel=1.0, n_views=96, n_bins=70, bin=1.0),
                               Geometry("fan", n=45, pixel=1.0, n_views=240, n_bins=90, bin=1.0, sod=150.0, sdd=250.0)],
                         ids=["parallel", "fan"])
def test_backprojection_single_axis_groups_match_general_path(air, torch_mod, g):
    """Groups of up to four images run eight views whose staged rays share one
    axis through a loop with no axis test (y-driven ones over horizontal pixel
    pairs, handed back through LDS); 8-image groups always take the general
    path.  Every pixel gets the same bits either way, also on tiles cut by the
    image edge (n = 45)."""
    plan = air.Plan(g, max_batch=8)
    axis, _, _ = plan.tables()
    groups = [set(np.unique(axis[v:v + 8]).tolist()) for v in range(0, g.n_views, 8)]
    assert {0} in groups and {1} in groups and {0, 1} in groups   # all three kinds of view group occur
    rng = np.random.default_rng(5)
    ys = rng.standard_normal((8, g.n_views, g.n_bins)).astype(np.float32)
    for filt in (0, 1):
        x8 = host(plan.filtered_backproject(dev(torch_mod, ys), filter=filt))
        x4 = host(plan.filtered_backproject(dev(torch_mod, ys[:4]), filter=filt))
        assert np.array_equal(x4, x8[:4]), filt
        for b in (0, 5):
            x1 = host(plan.filtered_backproject(dev(torch_mod, ys[b:b + 1]), filter=filt))[0]
            assert np.array_equal(x1, x8[b]), (filt, b)
    xs = rng.uniform(0, 0.03, (8, g.n, g.n)).astype(np.float32)
    z8 = host(plan.normal_apply(dev(torch_mod, xs), 0.5))
    z1 = host(plan.normal_apply(dev(torch_mod, xs[2:3]), 0.5))[0]
    assert np.array_equal(z1, z8[2])


def test_batch_above_plan_limit_is_rejected(air, torch_mod):
    plan = air.Plan(geom("small_par"), max_batch=1)
    x = torch_mod.zeros((2, 40, 40), device="cuda")
    with pytest.raises(air.AirError) as e:
        plan.project(x)
    assert e.value.status == air.AIR_E_INVALID


# ----------------------------------------------------------------------------- solver

def _oracle_solve(orc, g, y32, w, **kw):
    return orc.solve(orc.Geom(g), y32.astype(np.float64), w.lam, w.mu, w.n_outer, w.n_cg, **kw)


def test_solve_parity_c1(air, torch_mod, orc, record):
    w = synth.workload("c1")
    y = synth.make_case(w, 0)["y"].astype(np.float32)
    plan = air.Plan(w.geom)
    x, resid = plan.solve(dev(torch_mod, y[None]), w.lam, w.mu, w.n_outer, w.n_cg)
    xr, rr = _oracle_solve(orc, w.geom, y, w)
    record("rel_l2_final", rel(host(x)[0], xr))
    assert rel(host(x)[0], xr) < 1e-4
    np.testing.assert_allclose(host(resid)[0], rr, rtol=1e-3)


@pytest.mark.parametrize("filt", [0, 1])
def test_solve_l2_mode_and_ir_arm(air, torch_mod, orc, filt):
    w = synth.workload("c1")
    y = synth.make_case(w, 1)["y"].astype(np.float32)
    plan = air.Plan(w.geom)
    x, _ = plan.solve(dev(torch_mod, y[None]), 0.05, 1.0, 0, 8, reg=1, filter=filt, with_resid=False)
    xr, _ = orc.solve(orc.Geom(w.geom), y.astype(np.float64), 0.05, 1.0, 0, 8, reg=1, filter=filt)
    assert rel(host(x)[0], xr) < 1e-4
    # IR arm of the split Bregman solver
    x2, _ = plan.solve(dev(torch_mod, y[None]), w.lam, w.mu, 3, 4, filter=filt)
    xr2, _ = orc.solve(orc.Geom(w.geom), y.astype(np.float64), w.lam, w.mu, 3, 4, filter=filt)
    assert rel(host(x2)[0], xr2) < 1e-4


def test_solve_ragged_geometry(air, torch_mod, orc):
    g = RAGGED
    y = sino_for("ragged").astype(np.float32) * 0.1
    plan = air.Plan(g)
    x, _ = plan.solve(dev(torch_mod, y[None]), 0.01, 0.5, 4, 3)
    xr, _ = orc.solve(orc.Geom(g), y.astype(np.float64), 0.01, 0.5, 4, 3)
    assert rel(host(x)[0], xr) < 1e-4


def test_solve_degenerate_counts(air, torch_mod, orc):
    """n_outer = 0 leaves X untouched; n_cg = 0 runs only the Bregman updates."""
    w = synth.workload("c1")
    y = synth.make_case(w, 2)["y"].astype(np.float32)
    plan = air.Plan(w.geom)
    x0 = np.random.default_rng(3).uniform(0, 0.02, (1, 128, 128)).astype(np.float32)
    x, _ = plan.solve(dev(torch_mod, y[None]), w.lam, w.mu, 0, 5, x0=dev(torch_mod, x0))
    assert np.array_equal(host(x), x0.astype(np.float64))
    x, resid = plan.solve(dev(torch_mod, y[None]), w.lam, w.mu, 3, 0, x0=dev(torch_mod, x0))
    assert np.array_equal(host(x), x0.astype(np.float64))
    _, rr = orc.solve(orc.Geom(w.geom), y.astype(np.float64), w.lam, w.mu, 3, 0, x0=x0[0].astype(np.float64))
    np.testing.assert_allclose(host(resid)[0], rr, rtol=1e-4)


def test_solve_batch_invariance_and_determinism(air, torch_mod):
    """Each reconstruction is bit-identical alone, in a batch, and on a re-run."""
    w = synth.workload("c1", n_outer=4)
    ys = np.stack([synth.make_case(w, s)["y"] for s in range(3)]).astype(np.float32)
    plan = air.Plan(w.geom)
    xb, rb = plan.solve(dev(torch_mod, ys), w.lam, w.mu, w.n_outer, w.n_cg)
    xb2, _ = plan.solve(dev(torch_mod, ys), w.lam, w.mu, w.n_outer, w.n_cg)
    assert torch_mod.equal(xb, xb2)
    for b in range(3):
        x1, r1 = plan.solve(dev(torch_mod, ys[b:b + 1]), w.lam, w.mu, w.n_outer, w.n_cg)
        assert torch_mod.equal(x1[0], xb[b])
        assert torch_mod.equal(r1[0], rb[b])


@pytest.mark.parametrize("reg", [0, 1, 2])
def test_solve_split_batch_matches_single(air, torch_mod, reg):
    """Batches of 8 or more run as two sub-batches on two internal streams
    (6 + 5 images here): every image, start image and residual row is the same
    bits as its solve alone, and the call is ordered on the caller's stream
    (its input is written by a kernel on that stream just before the call)."""
    w = synth.workload("c1", n_outer=3)
    n = w.geom.n
    ys = np.stack([synth.make_case(w, s)["y"] for s in range(11)]).astype(np.float32)
    x0 = np.random.default_rng(5).uniform(0, 0.02, (11, n, n)).astype(np.float32)
    plan = air.Plan(w.geom)
    lam, mu = (w.lam, w.mu) if reg != 2 else (0.005, 1.0)
    side = torch_mod.cuda.Stream()
    with torch_mod.cuda.stream(side):
        Y = dev(torch_mod, ys) * 1.0           # written on `side`, read by the solve on `side`
        X0 = dev(torch_mod, x0) * 1.0
        xb, rb = plan.solve(Y, lam, mu, w.n_outer, w.n_cg, reg=reg, x0=X0)
        xb = xb * 1.0
    side.synchronize()
    for b in (0, 5, 6, 10):
        x1, r1 = plan.solve(dev(torch_mod, ys[b:b + 1]), lam, mu, w.n_outer, w.n_cg, reg=reg,
                            x0=dev(torch_mod, x0[b:b + 1]))
        assert torch_mod.equal(x1[0], xb[b]), b
        if reg != 1:
            assert torch_mod.equal(r1[0], rb[b]), b


@pytest.mark.parametrize("prec", ["mixed_f16", "mixed_bf16"])
def test_solve_mixed_precision_c1(air, torch_mod, orc, record, prec):
    w = synth.workload("c1")
    y = synth.make_case(w, 0)["y"].astype(np.float32)
    plan = air.Plan(w.geom, precision=prec)
    x, _ = plan.solve(dev(torch_mod, y[None]), w.lam, w.mu, w.n_outer, w.n_cg)
    xr, _ = _oracle_solve(orc, w.geom, y, w)
    record("rel_l2_final", rel(host(x)[0], xr))
    assert rel(host(x)[0], xr) < 1e-3


@pytest.mark.parametrize("case,wname", [("c2_fan_512_720_seed0", "c2"), ("c2_fan_512_180_seed0", "c2_25")])
def test_solve_parity_c2_full_size(air, torch_mod, record, case, wname):
    """512^2 fan beam, 50 Bregman x 5 CG, 720 and 180 views, against the stored
    oracle reconstruction (tests/golden/make_refs.py)."""
    path = os.path.join(HERE, "golden", case + ".npz")
    ref = np.load(path)
    w = synth.workload(wname)
    y = synth.make_case(w, 0)["y"].astype(np.float32)
    plan = air.Plan(w.geom)
    x, resid = plan.solve(dev(torch_mod, y[None]), w.lam, w.mu, w.n_outer, w.n_cg)
    record("rel_l2_final", rel(host(x)[0], ref["x"]))
    assert rel(host(x)[0], ref["x"]) < 1e-4
    np.testing.assert_allclose(host(resid)[0], ref["resid"], rtol=1e-2)


# ----------------------------------------------------------------------------- C3 and C5

def test_c3_batch64_precision_modes(air, torch_mod, orc, record):
    """64 seeded phantoms on the 128^2 parallel geometry in one batch: the ramp and
    A'^T per image in each precision mode, and final images of a subset."""
    from synth.phantom import batch_cases
    w = synth.workload("c3")
    _, ys = batch_cases(w, range(w.batch))
    ys = ys.astype(np.float32)
    G = orc.Geom(w.geom)
    ref_c = [orc.ramp(G, y.astype(np.float64)) for y in ys]
    ref_atc = [orc.filtered_backproject(G, y.astype(np.float64), 1) for y in ys]
    sub = range(0, 64, 8)
    ref_x = {i: orc.solve(G, ys[i].astype(np.float64), w.lam, w.mu, w.n_outer, w.n_cg)[0] for i in sub}
    Y = dev(torch_mod, ys)
    for prec, op_tol, final_tol in [("fp32", 1e-5, 1e-4), ("mixed_f16", 1e-5, 1e-3), ("mixed_bf16", 1e-5, 1e-3)]:
        plan = air.Plan(w.geom, max_batch=64, precision=prec)
        yf = host(plan.ramp(Y))
        xf = host(plan.filtered_backproject(Y, 1))
        ec = max(rel(yf[i], ref_c[i]) for i in range(64))
        ea = max(rel(xf[i], ref_atc[i]) for i in range(64))
        record(f"max_rel_l2_C_{prec}", ec)
        record(f"max_rel_l2_AtC_{prec}", ea)
        assert ec < op_tol and ea < op_tol, (prec, ec, ea)
        x, _ = plan.solve(Y, w.lam, w.mu, w.n_outer, w.n_cg, with_resid=False)
        x = host(x)
        ef = max(rel(x[i], ref_x[i]) for i in sub)
        record(f"max_rel_l2_final_{prec}", ef)
        assert ef < final_tol, (prec, ef)


@pytest.fixture(scope="module")
def c5_case():
    w = synth.workload("c5")
    return w, synth.make_case(w, 0)


def test_c5_operators_full_size(air, torch_mod, orc, record, c5_case):
    """1024^2 fan beam, 2304 views x 1536 bins: A and A'^T of one phantom."""
    w, case = c5_case
    g = w.geom
    plan = air.Plan(g, max_batch=1)
    G = orc.Geom(g)
    x = case["x_true"].astype(np.float32)
    y = host(plan.project(dev(torch_mod, x[None])))[0]
    e1 = rel(y, orc.project(G, x.astype(np.float64)))
    y32 = case["y"].astype(np.float32)
    xb = host(plan.filtered_backproject(dev(torch_mod, y32[None]), 1))[0]
    e2 = rel(xb, orc.filtered_backproject(G, y32.astype(np.float64), 1))
    record("rel_l2_A", e1)
    record("rel_l2_AtC", e2)
    assert e1 < 1e-5 and e2 < 1e-5, (e1, e2)


def test_c5_solve_against_stored_oracle(air, torch_mod, record, c5_case):
    """Two Bregman iterations (x 5 CG) of the 1024^2 case in a batch of two
    against the oracle's reconstruction stored by tests/golden/make_refs.py."""
    w, case = c5_case
    ref = np.load(os.path.join(HERE, "golden", "c5_fan_1024_2304_seed0_outer2.npz"))
    y = case["y"].astype(np.float32)
    plan = air.Plan(w.geom)
    Y = dev(torch_mod, np.stack([y, y[::-1].copy()]))
    x, resid = plan.solve(Y, w.lam, w.mu, 2, w.n_cg)
    e = rel(host(x)[0], ref["x"])
    record("rel_l2_final", e)
    assert e < 1e-4
    np.testing.assert_allclose(host(resid)[0], ref["resid"], rtol=1e-2)


# ----------------------------------------------------------------------------- forward-backward splitting

def _ir_step(air, torch_mod, g):
    from paper_1310_1434_amd import quality as Q
    plan = air.Plan(g)
    return 1.0 / Q.top_eigenvalue(plan, 0)


@pytest.mark.parametrize("name,filt", [("c1", 1), ("c1", 0), ("ragged", 1)])
def test_solve_fbs_parity(air, torch_mod, orc, record, name, filt):
    """Eq. (6) with the framelet proximal step: iterate and step-norm history
    against the oracle (AIR with A'^T, IR with A^T at step 1 / ||A^T A||)."""
    g = geom(name)
    y = sino_for(name, 2).astype(np.float32)
    mu = 1.0 if filt else _ir_step(air, torch_mod, g)
    plan = air.Plan(g)
    x, r = plan.solve(dev(torch_mod, y[None]), 0.005, mu, 15, 0, reg=2, filter=filt)
    xr, rr = orc.solve(orc.Geom(g), y.astype(np.float64), 0.005, mu, 15, 0, reg=2, filter=filt)
    record(f"rel_l2_fbs_{name}_{filt}", rel(host(x)[0], xr))
    assert rel(host(x)[0], xr) < 1e-4
    assert rel(r.cpu().numpy()[0], rr) < 1e-3


def test_solve_fbs_batch_invariance(air, torch_mod):
    g = geom("c1")
    plan = air.Plan(g)
    ys = np.stack([sino_for("c1", s) for s in range(3)]).astype(np.float32)
    xb, rb = plan.solve(dev(torch_mod, ys), 0.005, 1.0, 5, 0, reg=2)
    for b in range(3):
        x1, r1 = plan.solve(dev(torch_mod, ys[b:b + 1]), 0.005, 1.0, 5, 0, reg=2)
        assert np.array_equal(host(x1)[0], host(xb)[b])
        assert np.array_equal(r1.cpu().numpy()[0], rb.cpu().numpy()[b])


# ----------------------------------------------------------------------------- filtration variants

_VARIANTS = [("shepp-logan", False), ("hann", False), ("ram-lak", True), ("hann", True)]


def _flags(orc, ramp, cw):
    return orc.RAMP_WINDOWS[ramp] | (orc.RAMP_COSINE if cw else 0)


@pytest.mark.parametrize("prec", ["fp32", "mixed_f16", "mixed_bf16"])
@pytest.mark.parametrize("ramp,cw", _VARIANTS)
@pytest.mark.parametrize("name", ["ragged", "c1"])
def test_ramp_variant_parity(air, torch_mod, orc, record, name, ramp, cw, prec):
    """C = kappa D^(1/2) R D^(1/2) with the Shepp-Logan / Hann windows and the
    fan-beam cosine weighting (identity for the parallel-beam c1)."""
    g = geom(name)
    y = sino_for(name).astype(np.float32)
    plan = air.Plan(g, max_batch=1, precision=prec, ramp=ramp, cosine_weight=cw)
    og = orc.Geom(g, ramp=_flags(orc, ramp, cw))
    yf = host(plan.ramp(dev(torch_mod, y[None])))[0]
    e = rel(yf, orc.ramp(og, y.astype(np.float64)))
    record(f"rel_l2_C_{ramp}_{int(cw)}_{prec}", e)
    assert e < 1e-5, e
    if prec == "fp32":
        x = host(plan.filtered_backproject(dev(torch_mod, y[None]), filter=1))[0]
        assert rel(x, orc.filtered_backproject(og, y.astype(np.float64), 1)) < 1e-5


def test_variant_filtration_at_c2_and_in_a_solve(air, torch_mod, orc, record):
    """Hann window with cosine weighting: A'^T at full C2 size, and a split
    Bregman solve on the ragged fan geometry, against the oracle."""
    flags = _flags(orc, "hann", True)
    g = geom("c2")
    y = sino_for("c2").astype(np.float32)
    plan = air.Plan(g, ramp="hann", cosine_weight=True)
    x = host(plan.filtered_backproject(dev(torch_mod, y[None]), filter=1))[0]
    e = rel(x, orc.filtered_backproject(orc.Geom(g, ramp=flags), y.astype(np.float64), 1))
    record("rel_l2_AtC_c2_hann_cos", e)
    assert e < 1e-5
    g = geom("ragged")
    y = sino_for("ragged", 3).astype(np.float32)
    plan = air.Plan(g, ramp="hann", cosine_weight=True)
    xs, _ = plan.solve(dev(torch_mod, y[None]), 0.005, 1.0, 4, 4)
    xr, _ = orc.solve(orc.Geom(g, ramp=flags), y.astype(np.float64), 0.005, 1.0, 4, 4)
    assert rel(host(xs)[0], xr) < 1e-4


# ----------------------------------------------------------------------------- float16 image storage (mixed plans)

@pytest.mark.parametrize("name", ["ragged", "c2"])
@pytest.mark.parametrize("batch", [1, 3, 8])
def test_mixed_plan_projection_with_float16_images(air, torch_mod, orc, record, name, batch):
    """Mixed-precision plans store the projector's image copies in float16 with a
    per-image power-of-two scale (no overflow, no subnormals at these values):
    every sample carries a relative rounding error of at most the unit roundoff
    2^-11, and a projection of a nonnegative image is a sum of nonnegative terms,
    so its relative error stays below 2^-11 (plus float32 summation, ~1e-6); the
    bound is 5e-4.  An image's result is the same bits in any batch (its scale
    is its own, and its samples are summed in the same order)."""
    g = geom(name)
    rng = np.random.default_rng(batch)
    xs = np.stack([image_for(name, s) * rng.uniform(1e-3, 1e3) for s in range(batch)]).astype(np.float32)
    plan = air.Plan(g, max_batch=batch, precision="mixed_f16")
    y = host(plan.project(dev(torch_mod, xs)))
    for b in range(batch):
        e = rel(y[b], orc.project(orc.Geom(g), xs[b].astype(np.float64)))
        record(f"rel_l2_A_f16_{name}", e)
        assert e < 5e-4, (b, e)
        y1 = host(plan.project(dev(torch_mod, xs[b:b + 1])))[0]
        assert np.array_equal(y1, y[b])      # another grouping: same scale, same bits


def test_mixed_plan_projection_of_zero_and_tiny_images(air, torch_mod):
    g = geom("ragged")
    plan = air.Plan(g, max_batch=3, precision="mixed_f16")
    x = np.zeros((3, g.n, g.n), np.float32)
    x[1] = 1e-30 * np.random.default_rng(0).uniform(size=(g.n, g.n))
    x[2] = 1e30 * np.random.default_rng(1).uniform(size=(g.n, g.n))
    y = host(plan.project(dev(torch_mod, x)))
    assert np.all(y[0] == 0.0)
    # the float32 plan's reference for the 1e30 image is taken at 2^-40 of it
    # (float32 plans are specified below 2^80) and scaled back exactly
    s = np.array([1.0, 1.0, 2.0 ** -40], np.float32)[:, None, None]
    ref = host(air.Plan(g, max_batch=3).project(dev(torch_mod, x * s))) / s
    assert np.isfinite(y).all()
    assert rel(y[1], ref[1]) < 5e-4 and rel(y[2], ref[2]) < 5e-4


@pytest.mark.parametrize("prec", ["fp32", "mixed_f16"])
@pytest.mark.parametrize("reg", [0, 1])
def test_solve_commutes_with_power_of_two_scales(air, torch_mod, reg, prec):
    """Every float16 copy in a mixed solve takes a power-of-two scale relative to
    its own maximum: the image's from max |X|, each CG direction's from the
    bound max |r| + beta max |p_old| on max |p|, the split ramp's per row.  So a
    solve of 2^k Y is 2^k times the solve of Y, bit for bit, with sinograms of
    1e12 and 1e-12, far outside float16's range (split Bregman with 2^k lambda:
    its shrinkage threshold lambda / (2 mu) scales with the image; the L2
    problem's lambda weights X itself and stays).  The float32 path, specified
    below 2^80, does the same."""
    w = synth.workload("c1")
    y = np.stack([synth.make_case(w, s)["y"] for s in range(2)]).astype(np.float32)
    plan = air.Plan(w.geom, max_batch=2, precision=prec)
    lam = 0.05 if reg == 1 else w.lam
    n_outer, n_cg = (0, 8) if reg == 1 else (4, 4)

    def solve(k):
        f = 2.0 ** k
        lk = lam * f if reg == 0 else lam
        x, _ = plan.solve(dev(torch_mod, y * np.float32(f)), lk, w.mu, n_outer, n_cg, reg=reg, with_resid=False)
        return host(x)

    x0 = solve(0)
    assert np.isfinite(x0).all() and np.abs(x0).max() > 0
    for k in (40, -40):
        xk = solve(k)
        assert np.array_equal(xk, x0 * 2.0 ** k), k


@pytest.mark.parametrize("name", ["ragged", "c1"])
def test_float32_operators_commute_with_power_of_two_scales(air, torch_mod, name):
    """Within the float32 plans' range (below 2^80) the projector and the
    normal operator commute with power-of-two scaling bit for bit: the 2^32
    scale of the interpolation weights neither overflows nor changes a rounding,
    and tiny inputs keep their bits too."""
    g = geom(name)
    plan = air.Plan(g, max_batch=2)
    x = np.random.default_rng(5).uniform(0.0, 1.0, size=(2, g.n, g.n)).astype(np.float32)
    y0 = host(plan.project(dev(torch_mod, x)))
    n0 = host(plan.normal_apply(dev(torch_mod, x), 0.25))
    for k in (70, -70):
        f = np.float32(2.0 ** k)
        y = host(plan.project(dev(torch_mod, x * f)))
        assert np.array_equal(y, y0 * f), k
        nk = host(plan.normal_apply(dev(torch_mod, x * f), 0.25))
        assert np.array_equal(nk, n0 * f), k


@pytest.mark.parametrize("case,wname", [("c2_fan_512_720_seed0", "c2")])
def test_mixed_solve_c2_full_size(air, torch_mod, record, case, wname):
    """The mixed path (f16 hi/lo ramp and float16 image copies) at full C2 size
    against the stored oracle reconstruction, within the mixed bound 1e-3."""
    ref = np.load(os.path.join(HERE, "golden", case + ".npz"))
    w = synth.workload(wname)
    y = synth.make_case(w, 0)["y"].astype(np.float32)
    plan = air.Plan(w.geom, precision="mixed_f16")
    x, _ = plan.solve(dev(torch_mod, y[None]), w.lam, w.mu, w.n_outer, w.n_cg)
    e = rel(host(x)[0], ref["x"])
    record("rel_l2_final_mixed_c2", e)
    assert e < 1e-3


@pytest.mark.parametrize("prec", ["mixed_f16", "mixed_bf16"])
@pytest.mark.parametrize("scale", [1e-20, 1e20])
def test_split_ramp_at_extreme_sinogram_scales(air, torch_mod, orc, record, prec, scale):
    """The 16-bit splits keep float32-level accuracy at any sinogram scale: the
    float16 split takes a power-of-two scale per row from its max |y| (no
    overflow above 65504, no float16 subnormals for tiny rows), the bfloat16
    split has float32's exponent range.  C and A'^T = A^T C at 1e-20 and 1e+20
    times a C2 sinogram against the oracle."""
    g = geom("c2")
    y = (sino_for("c2") * scale).astype(np.float32)
    plan = air.Plan(g, max_batch=1, precision=prec)
    Y = dev(torch_mod, y[None])
    G = orc.Geom(g)
    yf = host(plan.ramp(Y))[0]
    e_c = rel(yf, orc.ramp(G, y.astype(np.float64)))
    x = host(plan.filtered_backproject(Y, filter=1))[0]
    e_a = rel(x, orc.filtered_backproject(G, y.astype(np.float64), 1))
    record(f"rel_l2_C_{prec}_scale{scale:g}", e_c)
    record(f"rel_l2_AtC_{prec}_scale{scale:g}", e_a)
    assert np.isfinite(yf).all() and np.isfinite(x).all()
    assert e_c < 1e-5 and e_a < 1e-5, (e_c, e_a)
