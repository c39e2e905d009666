"""GPU tests of the solve slots (air_state_*): continuous batching gives every
reconstruction the same bits as solving it alone, checkpoints resume exactly,
a broken slot does not disturb the others, and captured-graph steps match
eager steps at every replay."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

LAM, MU, NCG = 0.005, 1.0, 4


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1310_1434_amd import air
    w = synth.workload("c1")
    plan = air.Plan(w.geom, max_batch=1)
    ys = [torch.from_numpy(synth.make_case(w, s)["y"].astype(np.float32)).cuda() for s in range(5)]
    return torch, air, plan, ys


def solo(env, y, n_outer):
    torch, air, plan, _ = env
    x, r = plan.solve(y[None], LAM, MU, n_outer, NCG)
    torch.cuda.synchronize()
    return x[0].cpu().numpy(), r[0].cpu().numpy()


def finish(state, slot):
    x, r = state.retire(slot)
    state._torch_stream().synchronize()
    return x.cpu().numpy(), r.cpu().numpy()


def test_single_slot_matches_solve(env):
    torch, air, plan, ys = env
    st = air.State(plan, 2, LAM, MU, NCG, max_outer=6, stream=torch.cuda.Stream())
    s0 = st.admit(ys[0], n_outer=6)
    while st.query(s0)[0] < 6:
        assert st.step(2) == 2
    x, r = finish(st, s0)
    xs, rs = solo(env, ys[0], 6)
    assert np.array_equal(x, xs) and np.array_equal(r, rs)
    assert st.active == 0


def test_start_image_slot_matches_solve(env):
    """A slot admitted with a start image (whose carried residual g - M X0
    takes one operator apply at admission) gives the solve's bits, and a zero
    start image the same bits as none (M 0 = 0 exactly)."""
    torch, air, plan, ys = env
    x0 = torch.from_numpy(np.random.default_rng(5).uniform(0, 0.02, (128, 128)).astype(np.float32)).cuda()
    st = air.State(plan, 2, LAM, MU, NCG, max_outer=4, stream=torch.cuda.Stream())
    a = st.admit(ys[1], x0=x0, n_outer=4)
    z = st.admit(ys[1], x0=torch.zeros_like(x0), n_outer=4)
    while st.query(a)[0] < 4:
        st.step(4)
    xa, ra = finish(st, a)
    xz, rz = finish(st, z)
    xs, rs = plan.solve(ys[1][None], LAM, MU, 4, NCG, x0=x0[None].clone())
    torch.cuda.synchronize()
    assert np.array_equal(xa, xs[0].cpu().numpy()) and np.array_equal(ra, rs[0].cpu().numpy())
    xn, rn = solo(env, ys[1], 4)
    assert np.array_equal(xz, xn) and np.array_equal(rz, rn)


def test_continuous_batching_is_bit_identical_to_solo(env):
    """Requests join and leave between steps (slot ids are reused); every result
    equals its solo solve bit for bit."""
    torch, air, plan, ys = env
    st = air.State(plan, 3, LAM, MU, NCG, max_outer=8, stream=torch.cuda.Stream())
    n_outer = {0: 6, 1: 3, 2: 5, 3: 4}          # request (= sinogram index) -> iterations
    running = {}                               # request -> slot
    results = {}
    running[0] = st.admit(ys[0], n_outer=6)
    running[1] = st.admit(ys[1], n_outer=3)
    assert st.finished() == []
    assert st.step(10) == 3                    # limited by request 1
    assert st.finished() == [running[1]]       # air_state_poll: request 1 is through
    running[2] = st.admit(ys[2], n_outer=5)    # arrives while request 0 runs
    results[1] = finish(st, running.pop(1))    # its slot is freed; request 2 moves into its place
    running[3] = st.admit(ys[3], n_outer=4)    # reuses the freed slot id
    while running:
        assert st.step(1) == 1
        done = st.finished()
        for req, slot in list(running.items()):
            it, no = st.query(slot)
            assert no == n_outer[req]
            assert (slot in done) == (it == no)
            if it == no:
                results[req] = finish(st, running.pop(req))
    assert st.active == 0
    for req, n in n_outer.items():
        xs, rs = solo(env, ys[req], n)
        assert np.array_equal(results[req][0], xs), req
        assert np.array_equal(results[req][1], rs), req


def test_snapshot_resume_is_exact(env):
    torch, air, plan, ys = env
    stream = torch.cuda.Stream()
    st = air.State(plan, 1, LAM, MU, NCG, max_outer=6, stream=stream)
    s = st.admit(ys[4], n_outer=6)
    st.step(3)
    buf = st.snapshot(s)
    st.retire(s)
    st2 = air.State(plan, 2, LAM, MU, NCG, max_outer=6, stream=torch.cuda.Stream())
    s2 = st2.restore(buf)
    assert st2.query(s2) == (3, 6)
    st2.step(3)
    x, r = finish(st2, s2)
    xs, rs = solo(env, ys[4], 6)
    assert np.array_equal(x, xs) and np.array_equal(r, rs)


def _snapshot_x_and_c(buf, n, max_outer):
    """The image X and the carried residual c = A'^T Y - (A'^T A + mu I) X from a
    slot snapshot (header, X, c, b, d - b, residual history)."""
    np_ = n * n
    head = buf.size - 19 * np_ * 4 - max_outer * 8
    words = buf[head:head + 2 * np_ * 4].view(np.float32)
    return words[:np_].reshape(n, n), words[np_:].reshape(n, n)


@pytest.mark.parametrize("wname,prec,tol", [("c1", "fp32", 1e-5), ("c2", "fp32", 1e-5), ("c2", "mixed_f16", 1e-3)])
def test_carried_residual_tracks_the_true_one(wname, prec, tol, record):
    """After 50 Bregman iterations (250 CG steps) the residual a slot carries
    from one CG run to the next, c (updated by the CG recurrence instead of an
    operator apply), still equals A'^T Y - (A'^T A + mu I) X recomputed from the
    slot's X with the operators themselves, to the path's per-apply accuracy."""
    import torch
    from paper_1310_1434_amd import air
    w = synth.workload(wname)
    g = w.geom
    plan = air.Plan(g, max_batch=1, precision=prec)
    y = torch.from_numpy(synth.make_case(w, 1)["y"].astype(np.float32)).cuda()
    n_outer = 50
    st = air.State(plan, 1, w.lam, w.mu, w.n_cg, max_outer=n_outer, stream=torch.cuda.Stream())
    s = st.admit(y, n_outer=n_outer)
    while st.query(s)[0] < n_outer:
        st.step(n_outer)
    buf = st.snapshot(s)
    st.retire(s)
    x, c = _snapshot_x_and_c(buf, g.n, n_outer)
    xt = torch.from_numpy(x.copy()).cuda()[None]
    g_ = plan.filtered_backproject(y[None])
    c_true = (g_ - plan.normal_apply(xt, w.mu)).double().cpu().numpy()[0]
    torch.cuda.synchronize()
    err = np.linalg.norm(c.astype(np.float64) - c_true) / np.linalg.norm(g_.double().cpu().numpy())
    record(f"carried_residual_{wname}_{prec}", err)
    assert err < tol, err


def test_nonfinite_slot_is_isolated(env):
    """A slot whose sinogram holds a NaN: air_state_retire reports
    AIR_E_NONFINITE (and still copies it out and frees it); the other slot is
    untouched and retires with AIR_OK."""
    torch, air, plan, ys = env
    bad = ys[1].clone()
    bad[7, 11] = float("nan")
    st = air.State(plan, 2, LAM, MU, NCG, max_outer=3, stream=torch.cuda.Stream())
    g = st.admit(ys[0], n_outer=3)
    b = st.admit(bad, n_outer=3)
    st.step(3)
    with pytest.raises(air.NonFiniteResult) as e:
        st.retire(b)
    assert e.value.status == air.AIR_E_NONFINITE
    rb = e.value.resid.cpu().numpy()
    assert st.active == 1
    xg, rg = finish(st, g)
    assert not np.isfinite(rb).all()
    xs, rs = solo(env, ys[0], 3)
    assert np.array_equal(xg, xs) and np.array_equal(rg, rs)


def test_graph_replays_match_eager_steps(env):
    """Steps on a non-default stream replay a captured graph; compare every
    replay with eager steps on the default stream, with host synchronisation
    and other eager work in between."""
    torch, air, plan, ys = env
    eager = air.State(plan, 2, LAM, MU, NCG, max_outer=5)                           # default stream
    graph = air.State(plan, 2, LAM, MU, NCG, max_outer=5, stream=torch.cuda.Stream())
    se = [eager.admit(ys[k], n_outer=5) for k in (0, 2)]
    sg = [graph.admit(ys[k], n_outer=5) for k in (0, 2)]
    for _ in range(5):
        eager.step(1)
        graph.step(1)
        torch.cuda.synchronize()
        _ = plan.project(torch.rand((1, 128, 128), device="cuda"))    # unrelated eager work
        torch.cuda.synchronize()
        for a, b in zip(se, sg):
            ea, ga = eager.snapshot(a), graph.snapshot(b)
            assert np.array_equal(ea, ga)


def test_state_argument_checks(env):
    torch, air, plan, ys = env
    st = air.State(plan, 1, LAM, MU, NCG, max_outer=2)
    st.admit(ys[0], n_outer=2)
    with pytest.raises(air.AirError) as e:
        st.admit(ys[1], n_outer=2)                 # full
    assert e.value.status == air.AIR_E_NOMEM
    with pytest.raises(air.AirError):
        st.query(5)
    with pytest.raises(air.AirError):
        air.State(plan, 1, LAM, MU, NCG, max_outer=2).admit(ys[0], n_outer=3)   # above max_outer
