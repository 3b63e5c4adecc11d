"""Continuous-batching server for rigid registration requests.

A request is one observation/model pair registered by at most ``iters`` EM
iterations (Sec. 3.1 with the rigid twist M-step of Sec. 5), or fewer when the
engine stops it on a small twist (Sec. 6.1; the engine's twist_tol) or a
degenerate step.  The server keeps up to ``max_slots`` requests resident on the
device and advances all of them one EM iteration per tick with one batched
engine step; a request that arrives while others are running joins at the next
tick as soon as a slot, a range of the point arena and enough of the HBM budget
are free, and leaves (its slot, arena range and lattice freed) after its last
iteration.  Stopping is decided on the device: every tick the server enqueues
a read of the slots' states and retires the stopped ones when such a read has
completed, a tick or two later (the steps in between leave a stopped slot
unchanged).  The device side is the C engine (fr_engine_*); everything here is
scheduling.

The scheduling logic is written against a small backend interface so that it
can be exercised with a simulated device (``SimBackend``) as well as the GPU
(``EngineBackend``).
"""
from __future__ import annotations

import bisect
import collections
import gc
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

__all__ = ["Request", "Result", "ArenaAllocator", "Server", "SimBackend", "EngineBackend", "poisson_arrivals",
           "summarize"]


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds on the server clock
    m: int                         # model points
    n: int                         # observation points
    T0: np.ndarray = dataclasses.field(default_factory=lambda: np.eye(4))
    payload: object = None         # backend data (device clouds)


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    completed: float
    pose: np.ndarray
    status: int
    iterations: int = -1           # EM iterations the request ran (-1: not reported)

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of n requests at `rate` per second, first at 0."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    gaps[0] = 0.0
    return np.cumsum(gaps)


class ArenaAllocator:
    """First-fit allocator of point ranges in [0, capacity) with coalescing of freed ranges."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.free = [(0, self.capacity)]      # sorted (begin, length)

    def alloc(self, m: int) -> Optional[int]:
        m = max(int(m), 0)
        for i, (b, n) in enumerate(self.free):
            if n >= m:
                if n == m:
                    del self.free[i]
                else:
                    self.free[i] = (b + m, n - m)
                return b
        return None

    def release(self, b: int, m: int):
        if m <= 0:
            return
        i = bisect.bisect_left(self.free, (b, 0))
        self.free.insert(i, (b, m))
        # merge with the neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (self.free[i][0], self.free[i][1] + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]

    @property
    def free_points(self) -> int:
        return sum(n for _, n in self.free)


class Server:
    """Tick loop: admit (FIFO, as slots / arena / budget allow), step every resident request, retire.

    budget_bytes bounds the device bytes of the engine's lattices: a request is admitted only if the
    bytes in use plus the estimate ``bytes_per_obs_point * n`` of every request admitted in this tick
    stay within it.  max_inflight bounds how many ticks the host may run ahead of the device.
    """

    def __init__(self, backend, iters: int = 20, budget_bytes: int = 8 << 30, bytes_per_obs_point: float = 400.0,
                 max_admit: int = 32, max_inflight: int = 2):
        self.b = backend
        self.iters = int(iters)
        self.budget = int(budget_bytes)
        self.bpp = float(bytes_per_obs_point)
        self.max_admit = int(max_admit)
        self.max_inflight = int(max_inflight)
        self.arena = ArenaAllocator(backend.arena_points)
        self.ticks = 0
        self.max_resident = 0
        self.admit_calls = 0

    def _fits(self, req: Request, extra: float) -> bool:
        return self.b.usage() + extra + self.bpp * req.n <= self.budget

    def run(self, requests: Sequence[Request], on_tick: Optional[Callable] = None) -> List[Result]:
        # a collection of Python's oldest generation walks the whole host heap and stalls the tick loop
        # for tens of milliseconds (every request resident then waits); the objects alive at the start
        # are frozen out of the collector for the run, so collections only see what the run allocates
        gc.collect()
        gc.freeze()
        try:
            return self._run(requests, on_tick)
        finally:
            gc.unfreeze()

    def _run(self, requests: Sequence[Request], on_tick: Optional[Callable] = None) -> List[Result]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            if r.m > self.arena.capacity:
                raise ValueError(f"request {r.rid} has {r.m} model points, more than the arena holds")
            if self.bpp * r.n > self.budget:
                raise ValueError(f"request {r.rid} alone exceeds the HBM budget")
        nxt = 0                                   # next request not yet arrived
        queue: collections.deque = collections.deque()
        free_slots = list(range(self.b.max_slots - 1, -1, -1))
        active: Dict[int, list] = {}              # slot -> [request, steps enqueued, arena begin, admitted at]
        reads: collections.deque = collections.deque()   # (token, [(slot, request, admitted)]): final reads
        polls: collections.deque = collections.deque()   # (token, {slot: request id}): state reads
        ticks: collections.deque = collections.deque()   # tick tokens in flight
        results: List[Result] = []
        poll = bool(getattr(self.b, "stops_on_device", False))
        self.b.start()
        while nxt < len(reqs) or queue or active or reads:
            now = self.b.now()
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
            # admission, FIFO: stop at the first request that does not fit
            group, begins, slots = [], [], []
            extra = 0.0
            while queue and free_slots and len(group) < self.max_admit:
                r = queue[0]
                if not self._fits(r, extra):
                    break
                begin = self.arena.alloc(r.m)
                if begin is None:
                    break
                queue.popleft()
                extra += self.bpp * r.n
                group.append(r)
                begins.append(begin)
                slots.append(free_slots.pop())
            if group:
                self.b.admit(slots, group, begins)
                self.admit_calls += 1
                t_adm = self.b.now()
                for s, r, bgn in zip(slots, group, begins):
                    active[s] = [r, 0, bgn, t_adm]
            done = []
            if active:
                step_slots = sorted(active)
                self.b.step(step_slots)
                self.ticks += 1
                self.max_resident = max(self.max_resident, len(active))
                for s in step_slots:
                    active[s][1] += 1
                    if active[s][1] == self.iters:
                        done.append(s)
                if poll:
                    polls.append((self.b.read(poses=False), {s: active[s][0].rid for s in step_slots}))
            # slots the device has stopped, from the state reads that have completed
            while polls and self.b.done(polls[0][0]):
                token, snap = polls.popleft()
                state = self.b.states(token)
                for s, rid in snap.items():
                    if s in active and active[s][0].rid == rid and s not in done and state[s][2]:
                        done.append(s)
            if done:
                token = self.b.read()
                reads.append((token, [(s, active[s][0], active[s][3]) for s in done]))
                self.b.release(done)
                for s in done:
                    r, _, bgn, _ = active.pop(s)
                    self.arena.release(bgn, r.m)
                    free_slots.append(s)
            if active or group:
                ticks.append(self.b.mark())
                if on_tick is not None:
                    on_tick(self)
            # finished reads
            while reads and (self.b.done(reads[0][0]) or not active and not group):
                token, fin = reads.popleft()
                self.b.wait(token)
                t_done = self.b.completion_time(token)
                poses, state = self.b.poses(token)
                for s, r, t_adm in fin:
                    results.append(Result(r.rid, r.arrival, t_adm, t_done, poses[s].copy(), int(state[s][0]),
                                          int(state[s][1])))
            # keep the host at most max_inflight ticks ahead of the device
            while len(ticks) > self.max_inflight:
                self.b.wait(ticks.popleft())
            while ticks and self.b.done(ticks[0]):
                ticks.popleft()
            if not active and not group and not reads and nxt < len(reqs) and not queue:
                self.b.sleep_until(reqs[nxt].arrival)
        self.b.finish()
        results.sort(key=lambda x: x.rid)
        return results


def summarize(results: Sequence[Result], wall: Optional[float] = None) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    t0 = min(r.arrival for r in results)
    t1 = max(r.completed for r in results)
    span = (t1 - t0) if wall is None else wall
    return {"requests": len(results), "span_s": span, "registrations_per_s": len(results) / span,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "mean": float(lat.mean()), "max": float(lat.max())},
            "degenerate": int(sum(r.status != 0 for r in results)),
            "solved_per_s": sum(r.status == 0 for r in results) / span,
            "mean_iterations": float(np.mean([r.iterations for r in results]))}


# ------------------------------------------------------------------------------
class SimBackend:
    """A simulated device for testing the scheduler on the CPU: time advances by modelled durations
    (launch overhead + per-point cost), device bytes follow the modelled lattice sizes, and every
    step is logged so that a test can check what ran."""

    def __init__(self, max_slots=8, arena_points=10_000, step_fixed=1e-4, step_per_point=1e-8,
                 admit_fixed=5e-4, admit_per_point=2e-8, lattice_bytes_per_obs_point=300.0, fail=(),
                 stop_after=None):
        self.max_slots = max_slots
        # stop_after: request id -> the iteration after which the device stops it (its twist fell below
        # the tolerance); the server then learns of stops from state reads
        self.stop_after = dict(stop_after or {})
        self.stops_on_device = stop_after is not None
        self.arena_points = arena_points
        self.sf, self.sp, self.af, self.ap = step_fixed, step_per_point, admit_fixed, admit_per_point
        self.lbpp = lattice_bytes_per_obs_point
        self.fail = set(fail)              # request ids whose solve degenerates
        self.clock = 0.0                   # device-side completion time of the last queued work
        self.host = 0.0                    # host clock
        self.slots = {}                    # slot -> [request, begin, iterations]
        self.bytes = 0.0
        self.peak_bytes = 0.0
        self.log = []
        self.marks = []
        self.poses_at = []

    def start(self):
        pass

    def finish(self):
        self.host = max(self.host, self.clock)

    def now(self):
        return self.host

    def sleep_until(self, t):
        self.host = max(self.host, t)

    def usage(self):
        return self.bytes

    def admit(self, slots, reqs, begins):
        for s, r, b in zip(slots, reqs, begins):
            assert s not in self.slots, "slot admitted twice"
            for o, (rr, ob, _) in self.slots.items():
                assert b + r.m <= ob or ob + rr.m <= b, "arena ranges overlap"
            assert 0 <= b and b + r.m <= self.arena_points
            self.slots[s] = [r, b, 0]
            self.bytes += self.lbpp * r.n
        self.peak_bytes = max(self.peak_bytes, self.bytes)
        # the build runs on its own stream: the host waits for it, the device queue does not
        dur = self.af + self.ap * sum(r.n for r in reqs)
        self.host += dur
        self.log.append(("admit", tuple(slots), tuple(r.rid for r in reqs)))

    def _stopped(self, v):
        r, _, it = v
        return r.rid in self.fail and it >= 1 or it >= self.stop_after.get(r.rid, 1 << 30)

    def step(self, slots):
        for s in slots:
            if not self._stopped(self.slots[s]):      # a stopped slot is left unchanged
                self.slots[s][2] += 1
        pts = sum(self.slots[s][0].m for s in slots if not self._stopped(self.slots[s]))
        self.clock = max(self.clock, self.host) + self.sf + self.sp * pts
        self.host += 2e-5                  # enqueue cost
        self.log.append(("step", tuple(slots)))

    def read(self, poses=True):
        P = {s: np.array([[1.0, 0, 0, v[2]], [0, 1, 0, v[0].rid], [0, 0, 1, 0], [0, 0, 0, 1]])
             for s, v in self.slots.items()} if poses else None
        state = {s: (5 if v[0].rid in self.fail else 0, v[2], int(self._stopped(v))) for s, v in self.slots.items()}
        self.poses_at.append((self.clock, P, state))
        self.log.append(("read", poses))
        return len(self.poses_at) - 1

    def release(self, slots):
        for s in slots:
            r, _, _ = self.slots.pop(s)
            self.bytes -= self.lbpp * r.n
        self.log.append(("release", tuple(slots)))

    def mark(self):
        self.marks.append(self.clock)
        return ("tick", len(self.marks) - 1)

    def _time(self, token):
        return self.marks[token[1]] if isinstance(token, tuple) else self.poses_at[token][0]

    def done(self, token):
        return self._time(token) <= self.host

    def wait(self, token):
        self.host = max(self.host, self._time(token))

    def completion_time(self, token):
        return self._time(token)

    def poses(self, token):
        return self.poses_at[token][1], self.poses_at[token][2]

    def states(self, token):
        return self.poses_at[token][2]


class EngineBackend:
    """The GPU: an fr_engine on the current torch stream.  Completion times are read from timing
    events against a start event whose host time is known, so a latency is the device's, not that of
    the host's polling."""

    def __init__(self, ctx, params, payload_clouds: Callable):
        import torch
        from . import Engine, fr_ctx_usage
        self.torch = torch
        self.ctx = ctx
        self.eng = Engine(ctx, params)
        self.max_slots = int(params.max_slots)
        self.arena_points = int(params.arena_points)
        self.stops_on_device = float(params.twist_tol) > 0.0
        self.clouds = payload_clouds            # requests -> (model Cloud, obs Cloud) of len(requests) sets
        self._usage = fr_ctx_usage
        self.base = self.arena_bytes = 0
        self.pin_poses = []
        self.pin_status = []
        self.events = []
        self.read_ev = {}

    def start(self):
        torch = self.torch
        torch.cuda.synchronize()
        self.base = self._usage(self.ctx.h)
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record()
        torch.cuda.synchronize()
        self.t0_host = time.perf_counter()

    def finish(self):
        self.torch.cuda.synchronize()

    def now(self):
        return time.perf_counter() - self.t0_host

    def sleep_until(self, t):
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)

    def usage(self):
        return self._usage(self.ctx.h) - self.base

    def admit(self, slots, reqs, begins):
        model, obs = self.clouds(reqs)
        T0 = np.stack([r.T0 for r in reqs])
        self.eng.admit(slots, model, obs, begins, T0)

    def step(self, slots):
        self.eng.step(slots)

    def _pinned(self, kind):
        # pinned host buffers are reused once their read has been consumed (allocating pinned memory
        # every tick costs more host time than the tick itself)
        pool = self.pin_poses if kind == "poses" else self.pin_status
        if pool:
            return pool.pop()
        shape, dt = ((self.max_slots, 16), self.torch.float64) if kind == "poses" else \
            ((self.max_slots, 4), self.torch.int32)
        return self.torch.empty(shape, dtype=dt, pin_memory=True)

    def read(self, poses=True):
        torch = self.torch
        pp = self._pinned("poses") if poses else None
        ps = self._pinned("status")
        self.eng.read(pp, ps)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        self.read_ev[id(ev)] = (ev, pp, ps)
        return id(ev)

    def release(self, slots):
        self.eng.release(slots)

    def mark(self):
        ev = self.torch.cuda.Event()
        ev.record()
        return ev

    def done(self, token):
        ev = self.read_ev[token][0] if isinstance(token, int) else token
        return ev.query()

    def wait(self, token):
        ev = self.read_ev[token][0] if isinstance(token, int) else token
        ev.synchronize()

    def completion_time(self, token):
        ev = self.read_ev[token][0]
        return self.t0_event.elapsed_time(ev) / 1e3

    def poses(self, token):
        ev, pp, ps = self.read_ev.pop(token)
        out = pp.numpy().reshape(-1, 4, 4).copy(), ps.numpy().copy()
        self.pin_poses.append(pp)
        self.pin_status.append(ps)
        return out

    def states(self, token):
        ev, pp, ps = self.read_ev.pop(token)
        out = ps.numpy().copy()
        self.pin_status.append(ps)
        if pp is not None:
            self.pin_poses.append(pp)
        return out

    def close(self):
        self.eng.close()
