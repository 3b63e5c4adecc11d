"""Scheduling logic of the continuous-batching server, on a simulated device (no GPU)."""
import numpy as np
import pytest

from paper_1811_10136_amd.serve import ArenaAllocator, Request, Server, SimBackend, poisson_arrivals, summarize


def _stream(n=40, rate=2000.0, seed=0, lo=100, hi=3000):
    rng = np.random.default_rng(seed)
    t = poisson_arrivals(n, rate, seed)
    m = np.exp(rng.uniform(np.log(lo), np.log(hi), n)).astype(int)
    return [Request(i, float(t[i]), int(m[i]), int(m[i] * 0.95)) for i in range(n)]


def test_arena_allocator_first_fit_and_coalescing():
    a = ArenaAllocator(100)
    assert a.alloc(30) == 0 and a.alloc(30) == 30 and a.alloc(30) == 60
    assert a.alloc(20) is None
    a.release(30, 30)
    assert a.alloc(40) is None            # the hole is 30 wide, the tail 10
    a.release(0, 30)
    assert a.free == [(0, 60), (90, 10)]  # merged with its neighbour
    a.release(60, 30)
    assert a.free == [(0, 100)] and a.free_points == 100
    assert a.alloc(0) == 0 and a.free_points == 100


def test_poisson_driver_is_deterministic():
    a = poisson_arrivals(5000, 100.0, 3)
    b = poisson_arrivals(5000, 100.0, 3)
    np.testing.assert_array_equal(a, b)
    assert a[0] == 0.0 and np.all(np.diff(a) >= 0)
    assert abs(np.mean(np.diff(a)) - 0.01) < 0.001
    assert not np.array_equal(a, poisson_arrivals(5000, 100.0, 4))


def test_every_request_runs_exactly_its_iterations_under_the_limits():
    be = SimBackend(max_slots=6, arena_points=8000, lattice_bytes_per_obs_point=300.0)
    budget = 2_000_000
    srv = Server(be, iters=7, budget_bytes=budget, bytes_per_obs_point=300.0, max_admit=4)
    reqs = _stream()
    res = srv.run(reqs)
    assert [r.rid for r in res] == [r.rid for r in reqs]
    # per request: stepped exactly `iters` times between its admission and its release
    steps = {r.rid: 0 for r in reqs}
    slot_of = {}
    for ev in be.log:
        if ev[0] == "admit":
            for s, rid in zip(ev[1], ev[2]):
                assert s not in slot_of
                slot_of[s] = rid
        elif ev[0] == "step":
            assert len(ev[1]) <= 6
            for s in ev[1]:
                steps[slot_of[s]] += 1
        elif ev[0] == "release":
            for s in ev[1]:
                del slot_of[s]
    assert set(steps.values()) == {7}
    assert not slot_of
    assert be.peak_bytes <= budget
    # FIFO admission
    order = [rid for ev in be.log if ev[0] == "admit" for rid in ev[2]]
    assert order == sorted(order)
    # the recorded pose is the one the device held after the request's last step
    for r in res:
        assert r.pose[1, 3] == r.rid and r.pose[0, 3] == 7 and r.iterations == 7
        assert r.completed >= r.admitted >= r.arrival
    s = summarize(res)
    assert s["requests"] == len(reqs) and s["degenerate"] == 0
    assert s["latency_ms"]["p99"] >= s["latency_ms"]["p50"] > 0


def test_budget_and_arena_throttle_admission():
    # arena for two requests at a time, budget for three: never more than two resident
    be = SimBackend(max_slots=8, arena_points=2 * 3000)
    reqs = [Request(i, 0.0, 3000, 3000) for i in range(6)]
    srv = Server(be, iters=3, budget_bytes=3 * 3000 * 300, bytes_per_obs_point=300.0)
    res = srv.run(reqs)
    assert len(res) == 6 and srv.max_resident == 2
    be = SimBackend(max_slots=8, arena_points=100_000, lattice_bytes_per_obs_point=300.0)
    srv = Server(be, iters=3, budget_bytes=3 * 3000 * 300, bytes_per_obs_point=300.0)
    res = srv.run([Request(i, 0.0, 3000, 3000) for i in range(7)])
    assert len(res) == 7 and srv.max_resident == 3
    assert be.peak_bytes <= 3 * 3000 * 300


def test_a_failing_request_retires_without_disturbing_others():
    be = SimBackend(max_slots=4, arena_points=20_000, fail={5, 11})
    reqs = _stream(n=16, seed=2)
    res = Server(be, iters=4, budget_bytes=1 << 30).run(reqs)
    for r in res:
        assert r.status == (5 if r.rid in (5, 11) else 0)
        # a degenerate step stops the slot on the device: later steps leave it unchanged
        n = 1 if r.rid in (5, 11) else 4
        assert r.pose[1, 3] == r.rid and r.pose[0, 3] == n and r.iterations == n


def test_requests_larger_than_the_arena_or_budget_are_rejected():
    be = SimBackend(max_slots=2, arena_points=1000)
    with pytest.raises(ValueError):
        Server(be, iters=2).run([Request(0, 0.0, 1001, 10)])
    with pytest.raises(ValueError):
        Server(be, iters=2, budget_bytes=1000, bytes_per_obs_point=400.0).run([Request(0, 0.0, 10, 10)])


def test_idle_server_waits_for_arrivals_and_latency_reflects_queueing():
    # a slow device and a burst: the later requests of the burst wait for slots
    be = SimBackend(max_slots=1, arena_points=10_000, step_fixed=1e-3, step_per_point=0.0, admit_fixed=0.0,
                    admit_per_point=0.0)
    reqs = [Request(0, 0.0, 100, 100), Request(1, 0.0, 100, 100), Request(2, 1.0, 100, 100)]
    res = Server(be, iters=5, budget_bytes=1 << 30).run(reqs)
    lat = [r.latency for r in res]
    assert lat[0] == pytest.approx(5e-3, rel=0.05)
    assert lat[1] == pytest.approx(10e-3, rel=0.05)      # queued behind request 0
    assert lat[2] == pytest.approx(5e-3, rel=0.05)       # arrives to an idle server
    assert res[2].admitted >= 1.0


def test_requests_that_stop_on_the_device_retire_early():
    """Twist-stopped requests (Sec. 6.1): the device stops a slot after its request's stop iteration; the
    server learns of it from a state read a tick or two later, retires it, and reports the pose and the
    iteration count the device held at the stop.  The others run the cap."""
    reqs = _stream(n=24, seed=5)
    stop = {r.rid: 2 + r.rid % 5 for r in reqs if r.rid % 3 != 0}
    be = SimBackend(max_slots=5, arena_points=20_000, stop_after=stop)
    srv = Server(be, iters=9, budget_bytes=1 << 30, max_admit=3)
    res = srv.run(reqs)
    assert [r.rid for r in res] == [r.rid for r in reqs]
    for r in res:
        n = stop.get(r.rid, 9)
        assert r.iterations == n and r.pose[0, 3] == n and r.pose[1, 3] == r.rid
    # a stopped request leaves within a few ticks of its stop: fewer steps in all than the cap would take
    steps = sum(len(ev[1]) for ev in be.log if ev[0] == "step")
    assert steps < 9 * len(reqs)
    assert any(ev == ("read", False) for ev in be.log)
    # the same stream with the cap alone runs every request 9 iterations
    be2 = SimBackend(max_slots=5, arena_points=20_000)
    res2 = Server(be2, iters=9, budget_bytes=1 << 30, max_admit=3).run(reqs)
    assert all(r.iterations == 9 for r in res2)
    assert not any(ev[0] == "read" and ev[1] is False for ev in be2.log)
