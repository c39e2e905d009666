"""Continuous-batching reconstruction server over the solve slots.

Requests (a sinogram, its scan geometry and a Bregman iteration count) are
grouped by geometry; each group owns one plan, one slot state and one HIP
stream, so groups run concurrently on the device.  The loop, repeated until
every request is done:

  1. retire: in every group whose last step has completed, slots that reached
     their iteration count are copied out and freed;
  2. admit: pending requests that have arrived are admitted first come, first
     served into a free slot of their group; a group is opened when the HBM
     budget allows (idle empty groups are closed, and then plans without a group
     dropped, to make room); a request whose group could never fit the budget is
     rejected;
  3. step: every group with active slots and fewer than `depth` steps in
     flight (2 by default) enqueues one more Bregman iteration (one replay of
     its captured graph), so the next step is already queued behind the
     running one; no step is enqueued past a slot's last iteration (the
     library stops there), so a finished slot waits only for its own step.

So a request that arrives while others are on the GPU joins at the next step
of its group, and finished ones leave without waiting for the rest.  The
executor abstraction lets the same scheduler run on the GPU (GpuExecutor) or
on a simulated clock (tests).

HBM accounting: a group's slot state is charged while the group is open; a
geometry's plan (tables and operator scratch) is charged once, from its
creation until it is dropped, since it outlives the groups that use it.  The
tracked total equals the device bytes the executor holds.
"""
from __future__ import annotations

import dataclasses
import hashlib
import time
from collections import deque

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    geom: object                  # scan geometry (beam, n, pixel, n_views, n_bins, bin, sod, sdd, view_cos, view_sin)
    y: np.ndarray                 # [n_views, n_bins] float32 sinogram (host)
    n_outer: int
    arrival: float = 0.0          # seconds from the start of the run
    admitted: float | None = None
    finished: float | None = None
    x: np.ndarray | None = None   # result image (GpuExecutor)
    resid: np.ndarray | None = None
    error: str | None = None

    @property
    def latency(self) -> float | None:
        return None if self.finished is None else self.finished - self.arrival


def geometry_key(g) -> tuple:
    angles = np.concatenate([np.asarray(g.view_cos, np.float64), np.asarray(g.view_sin, np.float64)])
    return (g.beam, int(g.n), float(g.pixel), int(g.n_views), int(g.n_bins), float(g.bin),
            float(getattr(g, "sod", 0.0)), float(getattr(g, "sdd", 0.0)),
            hashlib.sha1(angles.tobytes()).hexdigest())


class Group:
    def __init__(self, key, geom, capacity: int, nbytes: int):
        self.key = key
        self.geom = geom
        self.capacity = capacity
        self.nbytes = nbytes
        self.slots: dict[int, Request] = {}     # slot -> request
        self.impl = None                        # executor-specific


class GpuExecutor:
    """Groups on the GPU: a State of `capacity` slots and a stream each, over
    one Plan per geometry (kept from its first use until dropped)."""

    def __init__(self, lam: float, mu: float, n_cg: int, max_outer: int, capacity: int,
                 precision: str = "fp32", device: str = "cuda:0"):
        import torch
        from . import air
        self.torch, self.air = torch, air
        self.lam, self.mu, self.n_cg, self.max_outer = lam, mu, n_cg, max_outer
        self.capacity, self.precision, self.device = capacity, precision, device
        self._plans = {}
        self._sizes = {}
        self._upload = None     # stream of the host-to-device sinogram copies

    def _sizes_of(self, key, geom):
        if key not in self._sizes:
            self._sizes[key] = self.air.workspace_sizes(geom, self.capacity, self.lam, self.mu, self.n_cg,
                                                        self.max_outer, precision=self.precision)
        return self._sizes[key]

    def plan(self, key, geom):
        if key not in self._plans:
            self._sizes_of(key, geom)
            self._plans[key] = self.air.Plan(geom, max_batch=1, precision=self.precision, device=self.device)
        return self._plans[key]

    def group_bytes(self, key, geom) -> int:
        """Device bytes of a group's slot state (its plan is charged separately)."""
        return self._sizes_of(key, geom)[1]

    def plan_bytes(self, key, geom) -> int:
        """Device bytes of the geometry's plan (tables and operator scratch)."""
        return self._sizes_of(key, geom)[0]

    def plan_resident(self, key) -> bool:
        return key in self._plans

    def drop_plan(self, key):
        self._plans.pop(key, None)

    def resident_bytes(self) -> int:
        """Device bytes of the plans already built (e.g. ahead of a run)."""
        return sum(self._sizes[k][0] for k in self._plans)

    def open(self, group: Group):
        stream = self.torch.cuda.Stream(device=self.device)
        state = self.air.State(self.plan(group.key, group.geom), self.capacity, self.lam, self.mu, self.n_cg,
                               self.max_outer, stream=stream)
        group.impl = {"state": state, "stream": stream, "events": deque()}

    def close(self, group: Group):
        group.impl["stream"].synchronize()
        group.impl = None

    def admit(self, group: Group, req: Request) -> int:
        """Queue the request's sinogram upload on a copy stream and its admission
        behind it on the group's stream; the host does not wait for either (nor
        for the group's step in flight)."""
        torch = self.torch
        if self._upload is None:
            self._upload = torch.cuda.Stream(device=self.device)
        st, gs = group.impl["state"], group.impl["stream"]
        host = torch.from_numpy(np.ascontiguousarray(req.y, np.float32)).pin_memory()
        with torch.cuda.stream(self._upload):
            y = torch.empty(host.shape, dtype=torch.float32, device=self.device)
            y.copy_(host, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self._upload)
        gs.wait_event(ev)
        group.impl.setdefault("staged", {})
        with torch.cuda.stream(gs):
            slot = st.admit(y, n_outer=req.n_outer)       # (keeps y alive for the group's stream)
        group.impl["staged"][slot] = host                # pinned source, alive until the slot retires
        return slot

    def in_flight(self, group: Group) -> int:
        """Steps of the group enqueued and not yet completed."""
        evs = group.impl["events"]
        while evs and evs[0].query():
            evs.popleft()
        return len(evs)

    def idle(self, group: Group) -> bool:
        return self.in_flight(group) == 0

    def step(self, group: Group) -> int:
        """Enqueue one Bregman iteration of the group's active slots; 0 if a slot
        has reached its iteration count (it must be retired first)."""
        k = group.impl["state"].step(1)
        if k:
            ev = self.torch.cuda.Event()
            ev.record(group.impl["stream"])
            group.impl["events"].append(ev)
        return k

    def progress(self, group: Group, slot: int) -> tuple[int, int]:
        return group.impl["state"].query(slot)

    def retire(self, group: Group, slot: int, req: Request):
        try:
            x, r = group.impl["state"].retire(slot)
        except self.air.NonFiniteResult as e:      # AIR_E_NONFINITE: copied out and freed
            x, r = e.x, e.resid
            req.error = "non-finite residual"
        group.impl["stream"].synchronize()
        group.impl.get("staged", {}).pop(slot, None)
        req.x = x.cpu().numpy()
        req.resid = r.cpu().numpy()


class Server:
    def __init__(self, executor, hbm_budget: int, capacity: int, clock=time.perf_counter, sleep=time.sleep,
                 depth: int = 2, max_active: int | None = None):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.capacity = capacity
        self.depth = depth
        # at most this many groups get new steps at a time, those whose oldest
        # active request arrived first (None: every group with work)
        self.max_active = max_active
        self.clock, self.sleep = clock, sleep
        self.groups: dict[tuple, Group] = {}
        self.pending: deque[Request] = deque()
        self.done: list[Request] = []
        self.used = executor.resident_bytes()      # plans built ahead of the run
        self.plans: dict[tuple, int] = {}           # resident plan -> its bytes (built by this server)
        self.steps = 0

    # ---------------------------------------------------------------- helpers
    def _fits_ever(self, key, geom) -> bool:
        return self.ex.group_bytes(key, geom) + self.ex.plan_bytes(key, geom) <= self.budget

    def _open(self, key, geom) -> Group | None:
        nbytes = self.ex.group_bytes(key, geom)
        pbytes = 0 if self.ex.plan_resident(key) else self.ex.plan_bytes(key, geom)
        if nbytes + pbytes > self.budget:
            return None
        while self.used + nbytes + pbytes > self.budget:
            idle = [g for g in self.groups.values() if not g.slots and self.ex.idle(g)]
            if idle:
                self._close(idle[0])
                continue
            spare = [k for k in self.plans if k not in self.groups and k != key]
            if not spare:
                return None
            self.ex.drop_plan(spare[0])
            self.used -= self.plans.pop(spare[0])
        g = Group(key, geom, self.capacity, nbytes)
        self.ex.open(g)
        self.groups[key] = g
        self.used += nbytes + pbytes
        if pbytes:
            self.plans[key] = pbytes
        return g

    def _close(self, g: Group):
        self.ex.close(g)
        self.used -= g.nbytes
        del self.groups[g.key]

    # ---------------------------------------------------------------- one pass
    def poll(self, now: float) -> bool:
        busy = False
        # 1. retire finished slots of groups whose last step completed
        for g in list(self.groups.values()):
            if not g.slots or not self.ex.idle(g):
                continue
            for slot, req in list(g.slots.items()):
                it, n_outer = self.ex.progress(g, slot)
                if it >= n_outer:
                    self.ex.retire(g, slot, req)
                    req.finished = self.clock() - self._t0
                    del g.slots[slot]
                    self.done.append(req)
                    busy = True
        # 2. admit arrived requests, first come first served within each group
        blocked = set()
        for req in list(self.pending):
            if req.arrival > now:
                break
            key = geometry_key(req.geom)
            if key in blocked:
                continue
            g = self.groups.get(key)
            if g is None:
                if not self._fits_ever(key, req.geom):
                    req.error = "does not fit the HBM budget"
                    self.pending.remove(req)
                    self.done.append(req)
                    continue
                g = self._open(key, req.geom)
                if g is None:
                    blocked.add(key)
                    continue
            if len(g.slots) >= g.capacity:
                blocked.add(key)
                continue
            slot = self.ex.admit(g, req)
            req.admitted = now
            g.slots[slot] = req
            self.pending.remove(req)
            busy = True
        # 3. keep up to `depth` steps in flight in every group with work (or in
        #    the max_active groups holding the oldest requests)
        work = [g for g in self.groups.values() if g.slots]
        if self.max_active is not None and len(work) > self.max_active:
            work.sort(key=lambda g: min((r.arrival, r.rid) for r in g.slots.values()))
            work = work[:self.max_active]
        for g in work:
            if self.ex.in_flight(g) < self.depth:
                if self.ex.step(g):
                    self.steps += 1
                    busy = True
        return busy

    def run(self, requests: list[Request], idle_sleep: float = 2e-4) -> list[Request]:
        """Serve `requests` (arrival times relative to the start); returns them when all are done."""
        self.pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        self.done = []
        self._t0 = self.clock()
        total = len(requests)
        while len(self.done) < total:
            now = self.clock() - self._t0
            if not self.poll(now):
                self.sleep(idle_sleep)
        return sorted(self.done, key=lambda r: r.rid)


class FakeExecutor:
    """Simulated executor for scheduler tests: a step of a group with k active
    slots takes step_cost(group, k) seconds of a simulated clock.  `held` is
    the memory it would hold: open groups' states plus resident plans."""

    def __init__(self, bytes_per_group, step_cost, bytes_per_plan=lambda geom: 0):
        self.bytes_per_group = bytes_per_group
        self.bytes_per_plan = bytes_per_plan
        self.step_cost = step_cost
        self.now = 0.0
        self.opened = []
        self.log = []
        self.plans = {}
        self.held = 0

    def clock(self):
        return self.now

    def sleep(self, dt):
        self.now += dt

    def group_bytes(self, key, geom):
        return self.bytes_per_group(geom)

    def plan_bytes(self, key, geom):
        return self.bytes_per_plan(geom)

    def plan_resident(self, key):
        return key in self.plans

    def drop_plan(self, key):
        self.held -= self.plans.pop(key)
        self.log.append(("drop_plan", key))

    def resident_bytes(self):
        return sum(self.plans.values())

    def open(self, g):
        if g.key not in self.plans:
            self.plans[g.key] = self.bytes_per_plan(g.geom)
            self.held += self.plans[g.key]
        self.held += self.bytes_per_group(g.geom)
        g.impl = {"done_at": deque(), "iters": {}, "next": 0}
        self.opened.append(g.key)

    def close(self, g):
        self.log.append(("close", g.key))
        self.held -= self.bytes_per_group(g.geom)
        g.impl = None

    def admit(self, g, req):
        slot = g.impl["next"]
        g.impl["next"] += 1
        g.impl["iters"][slot] = [0, req.n_outer]
        self.log.append(("admit", req.rid, self.now))
        return slot

    def in_flight(self, g):
        q = g.impl["done_at"]
        while q and q[0] <= self.now:
            q.popleft()
        return len(q)

    def idle(self, g):
        return self.in_flight(g) == 0

    def step(self, g):
        its = g.impl["iters"]
        if any(its[slot][0] >= its[slot][1] for slot in g.slots):
            return 0                          # a finished slot must be retired first
        for slot in g.slots:
            its[slot][0] += 1
        q = g.impl["done_at"]
        start = q[-1] if q and q[-1] > self.now else self.now
        q.append(start + self.step_cost(g, len(g.slots)))
        return 1

    def progress(self, g, slot):
        return tuple(g.impl["iters"][slot])

    def retire(self, g, slot, req):
        self.log.append(("retire", req.rid, self.now))
        del g.impl["iters"][slot]


def poisson_arrivals(rate: float, count: int, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a seeded Poisson process of `rate` requests per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def latency_stats(reqs: list[Request]) -> dict:
    lat = np.array([r.latency for r in reqs if r.latency is not None and r.error is None])
    if lat.size == 0:
        return {"count": 0}
    return {"count": int(lat.size), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}
