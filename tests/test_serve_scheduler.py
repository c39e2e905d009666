"""Scheduler logic of the continuous-batching server on a simulated clock (no GPU)."""
import numpy as np
import pytest

from paper_1310_1434_amd.serve import FakeExecutor, Request, Server, latency_stats, poisson_arrivals


class Geo:
    def __init__(self, n, views):
        self.beam, self.n, self.pixel, self.n_views, self.n_bins, self.bin = "fan", n, 1.0, views, n, 1.0
        self.sod, self.sdd = 500.0, 900.0
        a = 2 * np.pi * np.arange(views) / views
        self.view_cos, self.view_sin = np.cos(a), np.sin(a)


G1, G2 = Geo(32, 20), Geo(48, 30)


def make(rid, geo, n_outer, t):
    return Request(rid, geo, np.zeros((geo.n_views, geo.n_bins), np.float32), n_outer, arrival=t)


def server(budget=10, capacity=2, cost=0.01, per_slot=0.001):
    ex = FakeExecutor(lambda g: 1, lambda g, k: cost + per_slot * k)
    return ex, Server(ex, budget, capacity, clock=ex.clock, sleep=ex.sleep)


def test_all_requests_complete_first_come_first_served():
    ex, srv = server()
    reqs = [make(i, G1 if i % 2 else G2, 3, 0.005 * i) for i in range(10)]
    done = srv.run(reqs)
    assert [r.rid for r in done] == list(range(10))
    for r in done:
        assert r.error is None and r.finished >= r.arrival + 3 * 0.01
    for geo in (G1, G2):
        rids = [rid for kind, rid, _ in ex.log if kind == "admit" and reqs[rid].geom is geo]
        assert rids == sorted(rids)


def test_request_arriving_during_a_run_joins_before_it_ends():
    ex, srv = server(capacity=4)
    a, b = make(0, G1, 10, 0.0), make(1, G1, 2, 0.03)
    srv.run([a, b])
    assert 0.03 <= b.admitted < a.finished
    assert b.finished < a.finished          # leaves without waiting for a


def test_capacity_bounds_the_active_slots():
    ex, srv = server(capacity=2)
    reqs = [make(i, G1, 2, 0.0) for i in range(5)]
    srv.run(reqs)
    active, peak = 0, 0
    for kind, rid, t in sorted(ex.log[:], key=lambda e: (e[2], e[0] == "admit")):
        active += 1 if kind == "admit" else -1
        peak = max(peak, active)
    assert peak == 2


def test_budget_defers_a_second_geometry_until_the_first_group_is_idle():
    ex, srv = server(budget=1)
    reqs = [make(0, G1, 3, 0.0), make(1, G2, 3, 0.001), make(2, G1, 3, 0.002)]
    done = srv.run(reqs)
    assert all(r.error is None for r in done)
    t_close = [i for i, e in enumerate(ex.log) if e[0] == "close"]
    t_admit_g2 = [i for i, e in enumerate(ex.log) if e[0] == "admit" and e[1] == 1]
    assert t_close and t_admit_g2 and t_close[0] < t_admit_g2[0]
    assert done[1].admitted >= max(done[0].finished, done[2].finished) - 1e-12


def test_request_that_can_never_fit_is_rejected():
    ex = FakeExecutor(lambda g: 5 if g is G2 else 1, lambda g, k: 0.01)
    srv = Server(ex, 2, 2, clock=ex.clock, sleep=ex.sleep)
    done = srv.run([make(0, G1, 2, 0.0), make(1, G2, 2, 0.0)])
    assert done[0].error is None
    assert done[1].error == "does not fit the HBM budget" and done[1].finished is None


def test_latency_stats_and_arrivals():
    t = poisson_arrivals(40.0, 2000, seed=0)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 40.0) < 3.0
    ex, srv = server(capacity=8)
    reqs = [make(i, G1, 2, float(t[i])) for i in range(20)]
    st = latency_stats(srv.run(reqs))
    assert st["count"] == 20 and 0 < st["p50_s"] <= st["p99_s"] <= st["max_s"]


def test_tracked_bytes_equal_bytes_held():
    """A geometry's plan is charged once, from its creation until it is dropped;
    a group's state while the group is open.  After every pass of the loop the
    server's figure equals what the executor holds, also while groups close and
    plans are dropped to make room."""
    G3 = Geo(40, 24)
    ex = FakeExecutor(lambda g: 4, lambda g, k: 0.01, bytes_per_plan=lambda g: 1)
    srv = Server(ex, 6, 2, clock=ex.clock, sleep=ex.sleep)
    seen = []
    poll = srv.poll

    def checked(now):
        busy = poll(now)
        assert srv.used == ex.held <= srv.budget
        seen.append(srv.used)
        return busy

    srv.poll = checked
    reqs = [make(0, G1, 2, 0.0), make(1, G2, 2, 0.001), make(2, G3, 2, 0.002), make(3, G1, 2, 0.003)]
    done = srv.run(reqs)
    assert all(r.error is None for r in done)
    assert any(e[0] == "drop_plan" for e in ex.log)      # 4 (state) + 1 (plan) + 1 (other plan) > 6
    assert max(seen) <= 6


def test_nonfinite_result_is_reported_and_does_not_stop_the_loop():
    class Bad(FakeExecutor):
        def retire(self, g, slot, req):
            super().retire(g, slot, req)
            if req.rid == 1:
                req.error = "non-finite residual"
    ex = Bad(lambda g: 1, lambda g, k: 0.01)
    srv = Server(ex, 10, 2, clock=ex.clock, sleep=ex.sleep)
    done = srv.run([make(i, G1, 2, 0.0) for i in range(3)])
    assert [r.error for r in done] == [None, "non-finite residual", None]
    assert latency_stats(done)["count"] == 2


def test_steps_are_enqueued_ahead_but_never_past_a_slot_end():
    """With two steps in flight a group's next iteration is queued behind the
    running one, so a coarse polling loop no longer idles the group between
    steps; no step is ever enqueued beyond a slot's iteration count."""
    def finish_time(depth):
        ex = FakeExecutor(lambda g: 1, lambda g, k: 0.01)
        srv = Server(ex, 10, 2, clock=ex.clock, sleep=ex.sleep, depth=depth)
        peak = []
        poll = srv.poll

        def watched(now):
            busy = poll(now)
            for g in srv.groups.values():
                peak.append(ex.in_flight(g))
                for slot in g.slots:
                    it, n_outer = ex.progress(g, slot)
                    assert it <= n_outer
            return busy

        srv.poll = watched
        done = srv.run([make(0, G1, 6, 0.0), make(1, G1, 4, 0.0)], idle_sleep=0.004)
        return max(r.finished for r in done), max(peak)

    t1, p1 = finish_time(1)
    t2, p2 = finish_time(2)
    assert p1 == 1 and p2 == 2
    assert t2 < t1


def test_max_active_steps_the_groups_holding_the_oldest_requests():
    """With max_active groups stepping at a time, the group whose oldest request
    arrived first gets the steps; a later group waits until that request is
    done, then gets its turn (no group starves: every request completes)."""
    ex = FakeExecutor(lambda g: 1, lambda g, k: 0.01)
    srv = Server(ex, 10, 2, clock=ex.clock, sleep=ex.sleep, max_active=1)
    steps = []
    step = ex.step

    def logged(g):
        k = step(g)
        if k:
            steps.append((ex.now, g.key))
        return k

    ex.step = logged
    reqs = [make(0, G1, 5, 0.0), make(1, G2, 3, 0.001), make(2, G1, 2, 0.03)]
    done = srv.run(reqs, idle_sleep=0.002)
    assert all(r.error is None for r in done)
    keys = [k for _, k in steps]
    first_g2 = next(i for i, k in enumerate(keys) if k != keys[0])
    # G1 runs request 0's five iterations (request 2 joins it for one); then
    # G2's request, older than request 2, gets the steps; request 2 ends last
    assert first_g2 == 5 and keys[5:8] == [keys[5]] * 3 and keys[8:] == [keys[0]]
    assert done[2].finished > done[1].finished
    assert done[0].finished <= done[1].finished
    # without the limit both groups step from the start
    ex2 = FakeExecutor(lambda g: 1, lambda g, k: 0.01)
    srv2 = Server(ex2, 10, 2, clock=ex2.clock, sleep=ex2.sleep)
    done2 = srv2.run([make(0, G1, 5, 0.0), make(1, G2, 3, 0.001), make(2, G1, 2, 0.03)], idle_sleep=0.002)
    assert done2[1].finished < done[1].finished
