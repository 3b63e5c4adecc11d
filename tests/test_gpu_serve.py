"""The serving engine on the GPU: continuous batching gives every request the result it gets alone."""
import numpy as np
import pytest

import oracle
import synth
from _helpers import upload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [3000, 41000, 1200, 17000, 64000, 5000, 9000, 26000]
ITERS = 6


@pytest.fixture(scope="module")
def fr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1811_10136_amd as fr
    return fr


@pytest.fixture(scope="module")
def ctx(fr):
    c = fr.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def pairs():
    return [synth.depth_pair(100 + i, target_points=m) for i, m in enumerate(SIZES)]


def _T0(p):
    """A start near the ground truth: every request has support (from the identity the sparse requests
    see one plane or nothing, and point-to-plane on one plane is degenerate)."""
    return p.T_gt @ oracle.se3_exp(np.array([0.003, -0.002, 0.002, 0.004, 0.002, -0.003]))


def _alone(fr, ctx, p, iters=ITERS, fused=False):
    prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=iters, w=p.w, fixed=True, fused=fused)
    T, st, _ = fr.register(ctx, upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n]), prm, T0=_T0(p)[None])
    return T[0], int(st[0])


def _engine(fr, ctx, p0, slots=4, arena=150_000, fused=False, tol=0.0, graph=False):
    prm = fr.engine_params(6, "pt2pl", p0.sigma, p0.sigma_n, max_slots=slots, arena_points=arena, w=p0.w,
                           fused=fused, tol=tol, graph=graph)
    return fr.Engine(ctx, prm)


def _read(eng, S, with_state=False):
    poses = torch.empty((S, 16), dtype=torch.float64, pin_memory=True)
    state = torch.empty((S, 4), dtype=torch.int32, pin_memory=True)
    eng.read(poses, state)
    torch.cuda.synchronize()
    if with_state:
        return poses.numpy().reshape(S, 4, 4).copy(), state.numpy().copy()
    return poses.numpy().reshape(S, 4, 4).copy(), state.numpy()[:, 0].copy()


@pytest.mark.parametrize("mode", ["eager", "fused", "graph"])
def test_engine_mix_is_bitwise_the_pair_alone(fr, ctx, pairs, mode):
    """Requests join and leave at different ticks, reuse slots and arena ranges, and share every
    launch with different neighbours; each ends bitwise where fr_register leaves it alone (graph: every
    step replays a captured graph, admissions and reads in between)."""
    fused = mode == "fused"
    print(f"[serve] mix {mode}", flush=True)
    alone = [_alone(fr, ctx, p, fused=fused) for p in pairs]
    eng = _engine(fr, ctx, pairs[0], fused=fused, graph=mode == "graph")
    S = eng.max_slots
    # schedule: (tick, requests admitted at that tick into (slot, arena begin))
    admissions = {0: [(0, 0, 0), (1, 1, 10_000)], 2: [(2, 2, 65_000), (3, 3, 70_000)],
                  ITERS: [(4, 0, 0)], ITERS + 1: [(5, 1, 90_000)], ITERS + 3: [(6, 2, 100_000), (7, 3, 110_000)]}
    resident, results = {}, {}
    keep = []      # the model clouds stay alive until a later step has consumed them
    tick = 0
    while len(results) < len(pairs):
        for rid, slot, begin in admissions.get(tick, []):
            p = pairs[rid]
            keep.append(upload([p.model], [p.model_n]))
            eng.admit([slot], keep[-1], upload([p.obs], [p.obs_n]), [begin], _T0(p)[None])
            resident[slot] = [rid, 0]
        if resident:
            eng.step(sorted(resident))
            fin = []
            for slot in list(resident):
                resident[slot][1] += 1
                if resident[slot][1] == ITERS:
                    fin.append(slot)
            if fin:
                poses, status = _read(eng, S)
                for slot in fin:
                    results[resident[slot][0]] = (poses[slot], int(status[slot]))
                    del resident[slot]
                eng.release(fin)
        tick += 1
        assert tick < 100
    eng.close()
    for rid in range(len(pairs)):
        T_mix, st_mix = results[rid]
        T_alone, st_alone = alone[rid]
        assert st_mix == st_alone, rid
        np.testing.assert_array_equal(T_mix, T_alone, err_msg=f"request {rid}")
    assert sum(st == 0 for _, st in alone) >= len(pairs) - 1


def test_engine_result_matches_the_oracle(fr, ctx, pairs):
    p = pairs[5]
    eng = _engine(fr, ctx, p)
    model = upload([p.model], [p.model_n])
    eng.admit([2], model, upload([p.obs], [p.obs_n]), [500], _T0(p)[None])
    for _ in range(ITERS):
        eng.step([2])
    poses, status = _read(eng, eng.max_slots)
    eng.close()
    ref = oracle.register_rigid(p.model, p.model_n, p.obs, p.obs_n, feat=6, residual="pt2pl", sigma=p.sigma,
                                sigma_n=p.sigma_n, w=p.w, iters=ITERS, T0=_T0(p))
    assert status[2] == 0
    assert np.abs(poses[2] - ref).max() < 1e-4


def test_engine_rejects_bad_slot_and_arena_use(fr, ctx, pairs):
    p = pairs[0]
    eng = _engine(fr, ctx, p, slots=2, arena=10_000)
    m, o = upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n])
    T0 = _T0(p)[None]
    eng.admit([0], m, o, [0], T0)
    with pytest.raises(fr.FRError) as e:
        eng.admit([0], m, o, [5000], T0)          # slot occupied
    assert e.value.status == fr.FR_EINVAL
    with pytest.raises(fr.FRError):
        eng.admit([1], m, o, [len(p.model) - 1], T0)   # overlaps slot 0's range
    with pytest.raises(fr.FRError):
        eng.admit([1], m, o, [10_000 - len(p.model) + 1], T0)   # past the arena
    with pytest.raises(fr.FRError):
        eng.step([1])                                             # not occupied
    with pytest.raises(fr.FRError):
        eng.step([0, 0])                                          # repeated
    eng.step([0])
    eng.release([0])
    with pytest.raises(fr.FRError):
        eng.release([0])
    eng.admit([1], m, o, [len(p.model) - 1], T0)    # range free again
    eng.step([1])
    _, status = _read(eng, 2)
    assert status[1] == 0
    eng.close()


def test_server_on_the_gpu_matches_alone_runs(fr, ctx, pairs):
    """A small Poisson stream through the server: every result equals the pair alone, bitwise."""
    from paper_1811_10136_amd.serve import EngineBackend, Request, Server, poisson_arrivals, summarize
    reqs_p = [pairs[i % len(pairs)] for i in range(16)]
    model = fr.Cloud.from_numpy([p.model for p in reqs_p], [p.model_n for p in reqs_p])
    obs = fr.Cloud.from_numpy([p.obs for p in reqs_p], [p.obs_n for p in reqs_p])

    def clouds(reqs):
        a, b = reqs[0].rid, reqs[-1].rid + 1
        assert [r.rid for r in reqs] == list(range(a, b))
        return model.sets(a, b), obs.sets(a, b)

    prm = fr.engine_params(6, "pt2pl", pairs[0].sigma, pairs[0].sigma_n, max_slots=5, arena_points=160_000,
                           w=pairs[0].w)
    be = EngineBackend(ctx, prm, clouds)
    t = poisson_arrivals(len(reqs_p), 400.0, 7)
    reqs = [Request(i, float(t[i]), len(p.model), len(p.obs), T0=_T0(p)) for i, p in enumerate(reqs_p)]
    res = Server(be, iters=ITERS, budget_bytes=1 << 31, max_admit=3).run(reqs)
    be.close()
    alone = {}
    for r in res:
        k = r.rid % len(pairs)
        if k not in alone:
            alone[k] = _alone(fr, ctx, pairs[k])
        assert r.status == alone[k][1]
        np.testing.assert_array_equal(r.pose, alone[k][0], err_msg=f"request {r.rid}")
        assert r.completed > r.admitted >= r.arrival
    s = summarize(res)
    print(f"[serve] {s}", flush=True)


TOL = 2e-5


def _alone_tol(fr, ctx, p, iters=40):
    prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=iters, w=p.w, fixed=False, tol=TOL)
    T, st, rep = fr.register(ctx, upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n]), prm, T0=_T0(p)[None])
    return T[0], int(st[0]), rep.iterations


def test_engine_stops_a_slot_on_its_twist_as_the_pair_alone(fr, ctx, pairs):
    """With a twist tolerance, each slot stops on the device after the same step as fr_register on the
    pair alone (Sec. 6.1); steps that still list a stopped slot leave it bitwise unchanged, and its state
    reports the stop and the iteration count."""
    print("[serve] stop on twist", flush=True)
    sub = [pairs[i] for i in (0, 2, 5, 6)]
    alone = [_alone_tol(fr, ctx, p) for p in sub]
    assert min(a[2] for a in alone) < 40, [a[2] for a in alone]
    eng = _engine(fr, ctx, sub[0], slots=4, arena=150_000, tol=TOL)
    keep = []
    begin = 0
    for j, p in enumerate(sub):
        keep.append(upload([p.model], [p.model_n]))
        eng.admit([j], keep[-1], upload([p.obs], [p.obs_n]), [begin], _T0(p)[None])
        begin += len(p.model)
    for _ in range(45):                   # every slot listed in every step, stopped or not
        eng.step([0, 1, 2, 3])
    poses, state = _read(eng, 4, with_state=True)
    eng.close()
    for j, (T, st, it) in enumerate(alone):
        assert state[j, 0] == st and state[j, 1] == it and state[j, 2] == 1, (j, state[j], it)
        np.testing.assert_array_equal(poses[j], T, err_msg=f"slot {j}")


def test_server_with_device_stops_matches_alone_runs(fr, ctx, pairs):
    """The server retires twist-stopped requests from the slots' states: poses, statuses and iteration
    counts equal fr_register's on each pair alone with the same tolerance."""
    from paper_1811_10136_amd.serve import EngineBackend, Request, Server, poisson_arrivals
    reqs_p = [pairs[i % len(pairs)] for i in range(12)]
    model = fr.Cloud.from_numpy([p.model for p in reqs_p], [p.model_n for p in reqs_p])
    obs = fr.Cloud.from_numpy([p.obs for p in reqs_p], [p.obs_n for p in reqs_p])

    def clouds(reqs):
        a, b = reqs[0].rid, reqs[-1].rid + 1
        return model.sets(a, b), obs.sets(a, b)

    prm = fr.engine_params(6, "pt2pl", pairs[0].sigma, pairs[0].sigma_n, max_slots=5, arena_points=160_000,
                           w=pairs[0].w, tol=TOL)
    be = EngineBackend(ctx, prm, clouds)
    t = poisson_arrivals(len(reqs_p), 300.0, 9)
    reqs = [Request(i, float(t[i]), len(p.model), len(p.obs), T0=_T0(p)) for i, p in enumerate(reqs_p)]
    res = Server(be, iters=40, budget_bytes=1 << 31, max_admit=3).run(reqs)
    be.close()
    alone = {}
    for r in res:
        k = r.rid % len(pairs)
        if k not in alone:
            alone[k] = _alone_tol(fr, ctx, pairs[k])
        T, st, it = alone[k]
        assert r.status == st and r.iterations == it, (r.rid, r.status, r.iterations, st, it)
        np.testing.assert_array_equal(r.pose, T, err_msg=f"request {r.rid}")


def test_graph_replays_equal_the_eager_steps_every_tick(fr, ctx, pairs):
    """Two engines run the same schedule, one replaying captured graphs: after every step the poses, the
    statuses, the iteration counts and the stop flags of both agree bitwise (the resident set changes
    between replays: admissions, a stop on the twist, releases)."""
    engs = [_engine(fr, ctx, pairs[0], slots=4, tol=1e-6), _engine(fr, ctx, pairs[0], slots=4, tol=1e-6,
                                                                   graph=True)]
    plan = {0: [(0, 0, 0), (5, 1, 10_000)], 1: [(2, 2, 60_000)], 4: [(3, 3, 90_000)]}
    keep = []
    resident = set()
    for tick in range(12):
        for rid, slot, begin in plan.get(tick, []):
            p = pairs[rid]
            keep.append((upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n])))
            for eng in engs:
                eng.admit([slot], keep[-1][0], keep[-1][1], [begin], _T0(p)[None])
            resident.add(slot)
        if tick == 8:
            for eng in engs:
                eng.release([1])
            resident.discard(1)
        for eng in engs:
            eng.step(sorted(resident))
        (pa, sa), (pb, sb) = (_read(e, e.max_slots, with_state=True) for e in engs)
        for s in resident:
            np.testing.assert_array_equal(pa[s], pb[s], err_msg=f"tick {tick} slot {s}")
            np.testing.assert_array_equal(sa[s], sb[s], err_msg=f"tick {tick} slot {s}")
    for eng in engs:
        eng.close()
