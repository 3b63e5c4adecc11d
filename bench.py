"""Benchmark: batched rigid point-to-plane registration of depth-frame pairs on one MI355X.

One step = one fr_register call over a batch of B pairs (default 64): lattice
build of every observation, then 20 EM iterations of E-step (slice) and M-step
reduction -- by default in one fused kernel (FR_FUSED; --fused 0 runs them as
two kernels, and the line reports that form's step beside) -- and binary64
solve/update, all through the C ABI.  Inputs are resident in HBM before the
timed region starts.

Workload: 640x480 pinhole depth renders (fx = fy = 525) of 3 planes + 5
spheres (about 260k points with normals); observation = the scene after a
random motion (<= 10 deg, <= 0.05 m), 2 mm depth noise, 5% dropout; d = 6
features (position / 0.03 m, normal / 0.5), point-to-plane, sorted splat.

Then the served stream: 4096 rigid point-to-plane requests of log-uniform
size (1k-300k model points, drawn from depth renders like the above) arrive
as a Poisson stream and are registered (20 EM iterations each) either one at
a time by fr_register (the plain loop) or by the continuous-batching server
(fr_engine_*: every resident request advances one EM iteration per batched
step).  The arrival rate sweeps multiples of the plain loop's measured
capacity; the headline is the largest rate whose served p99 latency stays
under 100 ms.

Prints one JSON line: metric/value (E-step model points per second over the
whole batched step), registrations/s and p50/p99 latency of the served stream,
the roofline of the E-step kernel (algorithmic bytes / mean kernel time from
HIP events recorded on the launch stream during the timed steps), the plain
loop beside the server, and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
EST_BYTES_PER_POINT = 24 + 28          # model position + normal in, M0 + M1 + N out (binary32)
FUSED_BYTES_PER_POINT = 24             # fused slice + reduction: only the model point and normal move
PARTIAL_ROW_BYTES = 32 * 4             # fused: one binary32 partial row of the normal equations per tile
FUSED_TILE = 256                       # points per fused tile (the E-step tile)
TUNE_FUSED = 16                        # autotuner entries of the fused kernel: 16 + transform kind
VERTEX_BYTES = 16 + 4 * 7              # packed 6-coordinate key + 7 binary32 values
ITERS = 20
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "estep_depth64_counters.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _make(seed):
    return synth.depth_pair(seed)


def make_pairs(n, workers):
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_make, range(n)))


def kernel_source_hash():
    """Hash of the sources that decide the E-step kernel and the table it reads (the build lays it out)."""
    h = hashlib.sha256()
    for f in ("estep.hip", "fr_device.h", "fr_mstep.h", "lattice_build.hip"):
        h.update(open(os.path.join(ROOT, "paper_1811_10136_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(pairs_points, kernel):
    """HBM bytes per E-step launch from committed rocprofv3 counter runs, if they match this kernel."""
    try:
        prof = json.load(open(PROFILE_SUMMARY))
    except (OSError, ValueError):
        return None
    if (prof.get("kernel_source_hash") != kernel_source_hash() or prof.get("model_points") != pairs_points
            or prof.get("kernel") != kernel):
        return None
    return prof.get("hbm_bytes_per_launch")


CPU_ITERS = 10     # EM iterations of each CPU sample (the rate is per model-point iteration, build included)
CPU_REPS = 5


def _cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_one(pair, iters):
    """One oracle registration in this process (one BLAS thread): (seconds, stage timings)."""
    from threadpoolctl import threadpool_limits
    import oracle
    with threadpool_limits(limits=1):
        tm = {}
        t0 = time.perf_counter()
        oracle.register_rigid(pair.model, pair.model_n, pair.obs, pair.obs_n, feat=6, residual="pt2pl",
                              sigma=pair.sigma, sigma_n=pair.sigma_n, w=pair.w, iters=iters, T0=np.eye(4),
                              timings=tm)
        return time.perf_counter() - t0, tm


def cpu_baseline(pairs, iters=CPU_ITERS, reps=CPU_REPS):
    """The CPU oracle (C + NumPy float64, as written) on a bounded sample of the batch's pairs.

    One thread: the first pair, `reps` times (lattice build + `iters` EM iterations): median of the
    full registration, of the build, and of the per-iteration E-step and M-step.  All cores: one pair
    per process on every core of the host share (at most 16), all at once, `reps` times; the median
    wall time gives the aggregate rate.  Rates are model-point iterations per second, build included,
    like the GPU figure."""
    import multiprocessing as mp
    ncpu = os.cpu_count() or 1
    workers = max(1, min(16, ncpu, len(pairs)))
    one = [_oracle_one(pairs[0], iters) for _ in range(reps)]
    reg = float(np.median([t for t, _ in one]))
    build = float(np.median([tm["build"] for _, tm in one]))
    est = float(np.median([x for _, tm in one for x in tm["estep"]]))
    mst = float(np.median([x for _, tm in one for x in tm["mstep"]]))
    m0 = len(pairs[0].model)
    walls = []
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        list(ex.map(_oracle_one, pairs[:workers], [1] * workers))   # start the workers and load the oracle
        for _ in range(reps):
            t0 = time.perf_counter()
            list(ex.map(_oracle_one, pairs[:workers], [iters] * workers))
            walls.append(time.perf_counter() - t0)
    wall = float(np.median(walls))
    pts = sum(len(p.model) for p in pairs[:workers])
    return {"value": pts * iters / wall, "unit": "points/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} depth pairs of the batch ({pts} model points), one per process, each a lattice "
                      f"build + {iters} EM iterations, run together {reps} times (median wall {wall:.2f} s); "
                      f"single-threaded C + NumPy float64 per process",
            "nproc": ncpu, "cpu_model": _cpu_model(),
            "single_thread": {"value": m0 * iters / reg, "unit": "points/s", "cores": 1,
                              "sample": f"pair 0 ({m0} model points), {reps} runs, medians",
                              "registration_ms": reg * 1e3, "build_ms": build * 1e3,
                              "estep_ms_per_iter": est * 1e3, "mstep_ms_per_iter": mst * 1e3}}


def copy_reference(nbytes=256 << 20, reps=3):
    """Plain device-to-device copies of a known size, so a counter run over this process can scale
    its HBM byte counters (the copy moves exactly nbytes in and nbytes out per launch)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy reference: {reps} copies of {nbytes} bytes")


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Achievable HBM bandwidth: the best of `reps` device-to-device copies of `nbytes` (read + write
    bytes over the copy's time, HIP events on the copy's stream)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    return 2.0 * nbytes / best / 1e9


# ------------------------------------------------------------------------------
# served stream
SERVE_FRAMES = 64
SERVE_FRAME_POINTS = 300_000


def _make_frame(seed):
    return synth.depth_pair(seed, target_points=SERVE_FRAME_POINTS)


def make_request_stream(n, seed, workers):
    """Requests of log-uniform size in [1k, 300k] model points.  Request i is a sorted random
    subsample (m_i model points, m_i * N/M observation points, image order kept) of one of
    SERVE_FRAMES depth-frame pairs rendered at 300k points; the subsampling runs on the device
    with a seeded generator.  Returns the model and observation clouds (one set per request,
    resident in HBM) and the per-request point counts."""
    import math
    import torch
    import paper_1811_10136_amd as fr
    t = time.time()
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        frames = list(ex.map(_make_frame, range(10_000, 10_000 + SERVE_FRAMES)))
    log(f"rendered {len(frames)} frames for the request stream in {time.time() - t:.1f} s")
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(1000), math.log(300_000), n)).astype(np.int64)
    fid = rng.integers(0, SERVE_FRAMES, n)
    fm = [torch.from_numpy(np.ascontiguousarray(np.concatenate([f.model, f.model_n], 1).T)).cuda() for f in frames]
    fo = [torch.from_numpy(np.ascontiguousarray(np.concatenate([f.obs, f.obs_n], 1).T)).cuda() for f in frames]
    m = np.array([min(int(sizes[i]), fm[fid[i]].shape[1]) for i in range(n)], dtype=np.int64)
    k = np.array([min(max(1, int(round(m[i] * fo[fid[i]].shape[1] / fm[fid[i]].shape[1]))), fo[fid[i]].shape[1])
                  for i in range(n)], dtype=np.int64)
    mo = np.concatenate([[0], np.cumsum(m)])
    oo = np.concatenate([[0], np.cumsum(k)])
    M = torch.empty((6, int(mo[-1])), dtype=torch.float32, device="cuda")
    O = torch.empty((6, int(oo[-1])), dtype=torch.float32, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    for i in range(n):
        a, b = fm[fid[i]], fo[fid[i]]
        im = torch.randperm(a.shape[1], generator=g, device="cuda")[:m[i]].sort().values
        io = torch.randperm(b.shape[1], generator=g, device="cuda")[:k[i]].sort().values
        M[:, mo[i]:mo[i + 1]] = a[:, im]
        O[:, oo[i]:oo[i + 1]] = b[:, io]
    torch.cuda.synchronize()
    del fm, fo
    model = fr.Cloud(*[M[j] for j in range(6)], offsets=mo)
    obs = fr.Cloud(*[O[j] for j in range(6)], offsets=oo)
    return model, obs, m, k, (M, O)


def run_plain(fr, ctx, model, obs, arrivals, prm):
    """One request at a time through fr_register, in arrival order (the collector frozen as in the
    server's loop, so neither side pauses for a full collection of the host heap)."""
    import gc
    gc.collect()
    gc.freeze()
    try:
        return _run_plain(fr, ctx, model, obs, arrivals, prm)
    finally:
        gc.unfreeze()


def _run_plain(fr, ctx, model, obs, arrivals, prm):
    from paper_1811_10136_amd.serve import Result
    out = []
    t0 = time.perf_counter()
    for i, a in enumerate(arrivals):
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
            now = time.perf_counter() - t0
        T, st, _ = fr.register(ctx, model.sets(i, i + 1), obs.sets(i, i + 1), prm)
        out.append(Result(i, float(a), now, time.perf_counter() - t0, T[0], int(st[0])))
    return out


def run_served(fr, ctx, model, obs, m, k, arrivals, iters, eprm, budget, max_admit):
    from paper_1811_10136_amd.serve import EngineBackend, Request, Server
    be = EngineBackend(ctx, eprm, lambda reqs: (model.sets(reqs[0].rid, reqs[-1].rid + 1),
                                                obs.sets(reqs[0].rid, reqs[-1].rid + 1)))
    srv = Server(be, iters=iters, budget_bytes=budget, bytes_per_obs_point=400.0, max_admit=max_admit,
                 max_inflight=3)
    res = srv.run([Request(i, float(arrivals[i]), int(m[i]), int(k[i])) for i in range(len(arrivals))])
    be.close()
    return res, srv


def serve_bench(fr, ctx, args):
    from paper_1811_10136_amd.serve import poisson_arrivals, summarize
    t = time.time()
    model, obs, m, k, keep = make_request_stream(args.serve_requests, 5, args.workers)
    n = len(m)
    log(f"request stream: {n} requests, {int(m.sum())} model / {int(k.sum())} obs points, staged in "
        f"{time.time() - t:.1f} s")
    p0 = synth.depth_pair(0, target_points=1000)
    stop = args.serve_tol > 0.0
    prm = fr.register_params(6, "pt2pl", p0.sigma, p0.sigma_n, iters=args.iters, w=0.1, fixed=not stop,
                             tol=args.serve_tol if stop else 1e-6)
    eprm = fr.engine_params(6, "pt2pl", p0.sigma, p0.sigma_n, max_slots=args.serve_slots,
                            arena_points=args.serve_arena, w=0.1, tol=args.serve_tol if stop else 0.0)
    budget = int(args.serve_budget_gib * (1 << 30))
    # warm both paths
    run_plain(fr, ctx, model, obs, np.zeros(8), prm)
    run_served(fr, ctx, model, obs, m[:16], k[:16], np.zeros(16), args.iters, eprm, budget, args.serve_admit)
    # plain-loop capacity: the first requests back to back
    nc = min(n, args.serve_capacity_requests)
    t0 = time.perf_counter()
    run_plain(fr, ctx, model, obs, np.zeros(nc), prm)
    cap = nc / (time.perf_counter() - t0)
    log(f"plain loop capacity {cap:.1f} registrations/s ({nc} requests back to back)")
    served, served_graph, plain = [], [], []
    eprm_graph = fr.engine_params(6, "pt2pl", p0.sigma, p0.sigma_n, max_slots=args.serve_slots,
                                  arena_points=args.serve_arena, w=0.1, tol=args.serve_tol if stop else 0.0,
                                  graph=True)
    run_served(fr, ctx, model, obs, m[:16], k[:16], np.zeros(16), args.iters, eprm_graph, budget, args.serve_admit)
    for graph, dest, ep in ((False, served, eprm), (True, served_graph, eprm_graph)):
        for x in args.serve_lambdas:
            rate = x * cap
            arr = poisson_arrivals(n, rate, 11)
            t0 = time.perf_counter()
            res, srv = run_served(fr, ctx, model, obs, m, k, arr, args.iters, ep, budget, args.serve_admit)
            s = summarize(res)
            s.update({"lambda_x": x, "lambda_per_s": rate, "ticks": srv.ticks, "max_resident": srv.max_resident,
                      "wall_s": time.perf_counter() - t0, "graph": graph})
            dest.append(s)
            log(f"served{' graph' if graph else ''} lambda={x}x ({rate:.0f}/s): {s['registrations_per_s']:.1f} "
                f"reg/s, p50 {s['latency_ms']['p50']:.1f} ms, p99 {s['latency_ms']['p99']:.1f} ms, resident <= "
                f"{srv.max_resident}")
    for x in args.plain_lambdas:
        rate = x * cap
        arr = poisson_arrivals(n, rate, 11)
        s = summarize(run_plain(fr, ctx, model, obs, arr, prm))
        s.update({"lambda_x": x, "lambda_per_s": rate})
        plain.append(s)
        log(f"plain   lambda={x}x ({rate:.0f}/s): {s['registrations_per_s']:.1f} reg/s, p50 "
            f"{s['latency_ms']['p50']:.1f} ms, p99 {s['latency_ms']['p99']:.1f} ms")
    ok = [s for s in served + served_graph if s["latency_ms"]["p99"] < 100.0]
    head = max(ok, key=lambda s: (s["lambda_x"], s["registrations_per_s"])) if ok else None
    del keep
    return {
        "workload": f"{n} rigid point-to-plane requests, model points log-uniform in [1k, 300k] (sorted random "
                    f"subsamples of {SERVE_FRAMES} depth renders at 300k points), d=6, at most {args.iters} EM "
                    f"iterations each" + (f", stopped on a twist below {args.serve_tol:g}" if stop else "") +
                    ", Poisson arrivals",
        "requests": n, "model_points": int(m.sum()), "obs_points": int(k.sum()),
        "plain_capacity_per_s": cap, "served": served, "served_graph": served_graph, "plain": plain,
        "engine": {"max_slots": args.serve_slots, "arena_points": args.serve_arena,
                   "lattice_budget_gib": args.serve_budget_gib, "max_admit": args.serve_admit},
        "headline": None if head is None else {
            "lambda_x": head["lambda_x"], "registrations_per_s": head["registrations_per_s"],
            "solved_per_s": head["solved_per_s"], "degenerate": head["degenerate"], "graph": head["graph"],
            "p50_ms": head["latency_ms"]["p50"], "p99_ms": head["latency_ms"]["p99"],
            "rule": "largest swept arrival rate whose served p99 latency is under 100 ms (eager or graph-replayed "
                    "steps, the higher throughput at that rate)"},
        "degenerate_note": "requests ending FR_EDEGENERATE (singular normal equations, pose kept): the frames' "
                           "rigid motions of up to 10 degrees about the camera leave too little of the model "
                           "within the 3 cm kernel, often only one plane (rank 3); the same count in the served "
                           "and the plain runs, and the oracle reaches the same verdict on such frames",
    }


# ------------------------------------------------------------------------------
# the other workloads: single-pair times (latency and throughput context, not roofline)
def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts)), out


def other_workloads(fr, ctx, reps=5):
    out = {}
    # ellipsoid pair: 2000 points + 10% outliers, point-to-point, d = 3, 30 iterations
    p = synth.ellipsoid_pair(0)
    prm = fr.register_params(3, "pt2pt", p.sigma, iters=30, w=p.w, profile=True)
    m, o = fr.Cloud.from_numpy([p.model]), fr.Cloud.from_numpy([p.obs])
    ms, (T, st, rep) = _timed(lambda: fr.register(ctx, m, o, prm), reps)
    out["ellipsoid_pt2pt"] = {"model_points": len(p.model), "obs_points": len(p.obs), "iters": 30,
                              "registration_ms": ms, "build_ms": rep.build_ms,
                              "estep_ms_per_launch": rep.estep_ms / max(1, rep.estep_launches)}
    # one depth-frame pair: the single-pair latency of the batched workload
    p = synth.depth_pair(0)
    m, o = fr.Cloud.from_numpy([p.model], [p.model_n]), fr.Cloud.from_numpy([p.obs], [p.obs_n])
    for fused in (False, True):
        prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=20, w=p.w, profile=True, fused=fused)
        ms, (T, st, rep) = _timed(lambda: fr.register(ctx, m, o, prm), reps)
        out["depth_pt2pl" + ("_fused" if fused else "")] = {
            "model_points": len(p.model), "obs_points": len(p.obs), "iters": 20, "registration_ms": ms,
            "build_ms": rep.build_ms, "estep_ms_per_launch": rep.estep_ms / max(1, rep.estep_launches),
            "mstep_ms_per_iter": rep.mstep_ms / max(1, rep.iterations)}
    # articulated: 60k points, 20 capsule links, 32 DOF, 15 iterations
    p = synth.articulated_pair(1)
    t = p.extra["tree"]
    kt = fr.KinematicTree(t.parent, t.dof_offset, t.origin, t.axis)
    prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=p.iters, w=p.w, profile=True)
    m, o = fr.Cloud.from_numpy([p.model], [p.model_n]), fr.Cloud.from_numpy([p.obs], [p.obs_n])

    def art():
        th = p.extra["theta0"].copy()
        return fr.fr_register_articulated(ctx.h, m, p.extra["body_offsets"], o, kt, prm, th)
    ms, (st, rep) = _timed(art, reps)
    out["articulated_pt2pl"] = {"model_points": len(p.model), "obs_points": len(p.obs), "bodies": 20, "dof": 32,
                                "iters": p.iters, "registration_ms": ms, "build_ms": rep.build_ms}
    # node graph: 100k points, 512 nodes, 20 iterations
    p = synth.nodegraph_pair(0)
    e = p.extra
    g = fr.NodeGraph(e["nodes"], e["skin_idx"], e["skin_w"], e["edges"], 1.0)
    prm = fr.register_params(3, "pt2pt", p.sigma, iters=p.iters, w=p.w, profile=True)
    m, o = fr.Cloud.from_numpy([p.model]), fr.Cloud.from_numpy([p.obs])

    def ngr():
        T = np.repeat(np.eye(4)[None], len(e["nodes"]), 0)
        return fr.fr_register_nodegraph(ctx.h, m, o, g, prm, T)
    ms, (st, rep) = _timed(ngr, 3)
    out["nodegraph_pt2pt"] = {"model_points": len(p.model), "obs_points": len(p.obs), "nodes": len(e["nodes"]),
                              "iters": p.iters, "registration_ms": ms, "build_ms": rep.build_ms,
                              "pcg_iters_last": rep.solver_iters}
    out["updated_sigma"] = updated_sigma_workloads(fr, ctx)
    out["uncustomised_filter"] = uncustomised_filter_workloads(fr, ctx)
    out["descriptors"] = descriptor_workloads(fr, ctx)
    return out


def descriptor_workloads(fr, ctx, n_pairs=30, max_iters=30, tol=1e-5):
    """Registration by descriptors alone (Eq. 8; the global registration of Tab. 2): 30 objects of 12k
    points with 16-dimensional descriptors, seen from arbitrary poses with 30% occlusion and 30% clutter,
    started at the identity; success = mean alignment error below 5 mm.  Then the descriptor E-step
    alone at 8, 16 and 32 dimensions on a 200k-point object."""
    import torch
    rows = []
    for seed in range(n_pairs):
        p = synth.feature_pair(200 + seed, dim=16)
        e = p.extra
        m, o = fr.Cloud.from_numpy([p.model]), fr.Cloud.from_numpy([p.obs])
        mf = torch.from_numpy(e["model_feat"]).cuda()
        of = torch.from_numpy(e["obs_feat"]).cuda()
        prm = fr.register_params(3, "pt2pt", 0.01, iters=max_iters, w=p.w, tol=tol, fixed=False)

        def run():
            th = np.repeat(np.eye(4)[None], 1, 0)
            st, rep = fr.fr_register_features(ctx.h, m, mf, o, of, 16, e["sigma_f"], prm, th)
            return th, rep
        ms, (th, rep) = _timed(run, 3)
        rows.append((ms, rep.iterations, alignment_error(th[0], p.T_gt, p.model)))
    a = np.array(rows)
    res = {"pairs": n_pairs, "dim": 16, "model_points": 12000, "start": "identity; rotations uniform up to 180 deg",
           "success_below_5mm": int((a[:, 2] < 5e-3).sum()), "median_ms": float(np.median(a[:, 0])),
           "mean_iterations": float(a[:, 1].mean()), "median_error_m": float(np.median(a[:, 2]))}
    for dim in (8, 16, 32):
        p = synth.feature_pair(7, m=200_000, dim=dim)
        e = p.extra
        m, o = fr.Cloud.from_numpy([p.model]), fr.Cloud.from_numpy([p.obs])
        mf = torch.from_numpy(e["model_feat"]).cuda()
        of = torch.from_numpy(e["obs_feat"]).cuda()
        prm = fr.register_params(3, "pt2pt", 0.01, iters=1, w=p.w, profile=True)

        def run():
            th = np.repeat(np.eye(4)[None], 1, 0)
            return fr.fr_register_features(ctx.h, m, mf, o, of, dim, e["sigma_f"], prm, th)[1]
        reps = [run() for _ in range(4)][1:]
        est = float(np.median([r.estep_ms for r in reps]))
        res[f"estep_dim{dim}"] = {"model_points": len(p.model), "obs_points": len(p.obs), "estep_ms": est,
                                  "model_points_per_s": len(p.model) / est * 1e3,
                                  "build_ms": float(np.median([r.build_ms for r in reps]))}
    return res


def uncustomised_filter_workloads(fr, ctx, n_pairs=8, max_iters=60, tol=1e-4):
    """The customised filter (lattice of Y built once, no blur) against the uncustomised one (joint
    lattice of Y and the moved X, blurred, rebuilt every iteration): the ellipsoid sweep of
    updated_sigma_workloads and one 640x480 depth frame, 20 iterations from near the ground truth."""
    rows = {"customised": [], "uncustomised": []}
    for seed in range(n_pairs):
        p = synth.ellipsoid_pair(100 + seed, max_angle_deg=10.0, max_trans=0.05, noise=0.01)
        m, o = fr.Cloud.from_numpy([p.model]), fr.Cloud.from_numpy([p.obs])
        for name, blurred in (("customised", False), ("uncustomised", True)):
            prm = fr.register_params(3, "pt2pt", p.sigma, iters=max_iters, w=p.w, tol=tol, fixed=False,
                                     blurred=blurred)
            ms, (T, st, rep) = _timed(lambda: fr.register(ctx, m, o, prm), 3)
            rows[name].append((rep.iterations, ms, alignment_error(T[0], p.T_gt, p.model)))
    res = {"pairs": n_pairs, "start": "identity; motions up to 10 deg, 5 cm", "noise": 0.01, "sigma": 0.02,
           "stop": f"twist below {tol} or {max_iters} iterations"}
    for k, v in rows.items():
        a = np.array(v)
        res[k] = {"mean_iterations": float(a[:, 0].mean()), "mean_ms": float(a[:, 1].mean()),
                  "mean_error_m": float(a[:, 2].mean()), "converged_below_5mm": int((a[:, 2] < 5e-3).sum())}
    p = synth.depth_pair(0)
    m, o = fr.Cloud.from_numpy([p.model], [p.model_n]), fr.Cloud.from_numpy([p.obs], [p.obs_n])
    for name, blurred in (("customised", False), ("uncustomised", True)):
        prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=20, w=p.w, profile=True, blurred=blurred)
        ms, (T, st, rep) = _timed(lambda: fr.register(ctx, m, o, prm), 3)
        res["depth_pt2pl_20_iters_" + name] = {
            "model_points": len(p.model), "obs_points": len(p.obs), "registration_ms": ms,
            "build_ms_total": rep.build_ms, "estep_ms_per_launch": rep.estep_ms / max(1, rep.estep_launches),
            "error_m": alignment_error(T[0], p.T_gt, p.model)}
    return res


def updated_sigma_workloads(fr, ctx, n_pairs=8, max_iters=60, tol=1e-4):
    """Fixed against updated sigma (Sec. 3.3, the two rows of Tab. 1): ellipsoid pairs (2000 points,
    10% outliers, noise 0.01) under motions up to 10 deg / 5 cm from the identity, run until the
    twist drops below `tol`; and one 640x480 depth frame, 20 iterations of the updated-sigma loop."""
    rows = {"fixed": [], "updated": []}
    for seed in range(n_pairs):
        p = synth.ellipsoid_pair(100 + seed, max_angle_deg=10.0, max_trans=0.05, noise=0.01)
        m, o = fr.Cloud.from_numpy([p.model]), fr.Cloud.from_numpy([p.obs])
        prm = fr.register_params(3, "pt2pt", p.sigma, iters=max_iters, w=p.w, tol=tol, fixed=False)
        ms, (T, st, rep) = _timed(lambda: fr.register(ctx, m, o, prm), 3)
        rows["fixed"].append((rep.iterations, ms, alignment_error(T[0], p.T_gt, p.model)))
        prm = fr.register_params(3, "pt2pt", p.sigma, iters=max_iters, w=p.w, tol=tol, fixed=False, m2=True)
        ms, (T, s, st, rep) = _timed(lambda: fr.register_sigma(ctx, m, o, prm, p.sigma[0], 1e-3), 3)
        rows["updated"].append((rep.iterations, ms, alignment_error(T[0], p.T_gt, p.model)))
    res = {"pairs": n_pairs, "start": "identity; motions up to 10 deg, 5 cm", "noise": 0.01, "sigma0": 0.02,
           "stop": f"twist below {tol} or {max_iters} iterations"}
    for k, v in rows.items():
        a = np.array(v)
        res[k] = {"mean_iterations": float(a[:, 0].mean()), "mean_ms": float(a[:, 1].mean()),
                  "mean_error_m": float(a[:, 2].mean()), "converged_below_5mm": int((a[:, 2] < 5e-3).sum())}
    p = synth.depth_pair(0)
    m, o = fr.Cloud.from_numpy([p.model], [p.model_n]), fr.Cloud.from_numpy([p.obs], [p.obs_n])
    prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=20, w=p.w, profile=True, m2=True)
    ms, (T, s, st, rep) = _timed(lambda: fr.register_sigma(ctx, m, o, prm, p.sigma[0], 2e-3), 3)
    res["depth_pt2pl_20_iters"] = {"model_points": len(p.model), "obs_points": len(p.obs), "registration_ms": ms,
                                   "rebuild_ms_per_iter": rep.build_ms / 20, "estep_ms_per_launch":
                                   rep.estep_ms / max(1, rep.estep_launches), "final_sigma": float(s[0])}
    return res


def batch_outcome(pairs, T, status):
    """How the registrations of the batch ended: solved to within 5 mm of the ground truth, or with
    singular normal equations (FR_EDEGENERATE).  The workload's rigid motions of up to 10 degrees about
    the camera move points 3 m away by up to 50 cm, against a 3 cm kernel; where too few model points
    then find support the Gauss-Newton system is singular (the oracle reaches the same verdict)."""
    err = [alignment_error(T[i], p.T_gt, p.model) for i, p in enumerate(pairs)]
    ok = [i for i in range(len(pairs)) if status[i] == 0]
    return {"pairs": len(pairs), "degenerate": int(sum(status != 0)),
            "within_5mm": int(sum(err[i] < 5e-3 for i in ok)),
            "median_error_m": float(np.median([err[i] for i in ok])) if ok else None}


def alignment_error(T, T_gt, x):
    """Mean |(T - T_gt) x| over the model points (Eq. 22)."""
    D = np.asarray(T) - np.asarray(T_gt)
    return float(np.mean(np.linalg.norm(np.asarray(x, np.float64) @ D[:3, :3].T + D[:3, 3], axis=1)))


def profile_workload(name):
    """One of the single-pair workloads alone, three times (the subject of a kernel trace)."""
    import torch
    import paper_1811_10136_amd as fr
    ctx = fr.Context(0)
    if name == "nodegraph":
        p = synth.nodegraph_pair(0)
        e = p.extra
        g = fr.NodeGraph(e["nodes"], e["skin_idx"], e["skin_w"], e["edges"], 1.0)
        prm = fr.register_params(3, "pt2pt", p.sigma, iters=p.iters, w=p.w)
        m, o = fr.Cloud.from_numpy([p.model]), fr.Cloud.from_numpy([p.obs])
        run = lambda: fr.fr_register_nodegraph(ctx.h, m, o, g, prm, np.repeat(np.eye(4)[None], len(e["nodes"]), 0))
    elif name == "articulated":
        p = synth.articulated_pair(1)
        t = p.extra["tree"]
        kt = fr.KinematicTree(t.parent, t.dof_offset, t.origin, t.axis)
        prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=p.iters, w=p.w)
        m, o = fr.Cloud.from_numpy([p.model], [p.model_n]), fr.Cloud.from_numpy([p.obs], [p.obs_n])
        run = lambda: fr.fr_register_articulated(ctx.h, m, p.extra["body_offsets"], o, kt, prm,
                                                 p.extra["theta0"].copy())
    elif name == "descriptors":
        p = synth.feature_pair(7, m=200_000, dim=16)
        e = p.extra
        m, o = fr.Cloud.from_numpy([p.model]), fr.Cloud.from_numpy([p.obs])
        mf, of = torch.from_numpy(e["model_feat"]).cuda(), torch.from_numpy(e["obs_feat"]).cuda()
        prm = fr.register_params(3, "pt2pt", 0.01, iters=20, w=p.w)
        run = lambda: fr.fr_register_features(ctx.h, m, mf, o, of, 16, e["sigma_f"], prm,
                                              np.repeat(np.eye(4)[None], 1, 0))
    else:
        p = synth.depth_pair(0)
        m, o = fr.Cloud.from_numpy([p.model], [p.model_n]), fr.Cloud.from_numpy([p.obs], [p.obs_n])
        if name == "uncustomised":
            prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=20, w=p.w, blurred=True)
            run = lambda: fr.register(ctx, m, o, prm)
        else:
            prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=20, w=p.w, m2=True)
            run = lambda: fr.register_sigma(ctx, m, o, prm, p.sigma[0], 2e-3)
    for i in range(3):
        run()
        torch.cuda.synchronize()
        log(f"{name}: run {i + 1} of 3 done")
    ctx.close()


BUILD_IN_BYTES = 24                        # observation position + normal in (binary32)
BUILD_VERTEX_BYTES = 16 + 4 + 4 * 8        # vertex out: packed key, occupancy, 7 values padded to 8 (binary32)
TABLE_SLOT_BYTES = 64                      # lookup table: key + padded values per slot, 2 slots per vertex
# bytes a partial record moves through the sorted build: written by the partial pass (key 16, count 4,
# values 28), key read by the insertion (16), (vertex, record) pair written and read (16), three radix
# passes over the pairs (3 x 16), count and values read by the per-vertex sums (32)
PARTIAL_BYTES_SORTED = 48 + 16 + 16 + 48 + 32
ATOMICS_PER_PARTIAL = 8                    # 7 binary32 value atomics + 1 occupancy atomic


def build_rates(fr, ctx, obs, sigma, sigma_n, reps=3):
    """Lattice build of the 64 observation frames, sorted and atomic splat: observation points per second,
    stage times, the algorithmic bytes of the build against HBM, the partial records' own traffic, and the
    atomic splat's value stage against the uncontended-atomic probe."""
    res = {}
    for name, splat in (("sorted", fr.FR_SPLAT_SORTED), ("atomic", fr.FR_SPLAT_ATOMIC)):
        prm = fr.lattice_params(6, 7, sigma, sigma_n, splat)
        ms, _ = _timed(lambda: fr.Lattice(ctx, obs, prm).close(), reps)
        stages = []
        for _ in range(reps):
            lat = fr.Lattice(ctx, obs, prm)
            stages.append(fr.fr_lattice_build_times(lat.h))
            inc, part = fr.fr_lattice_records(lat.h)
            nv = sum(lat.stats(s)[0] for s in range(obs.n_sets))
            lat.close()
        st = np.median(np.array(stages), axis=0)
        alg = obs.n * BUILD_IN_BYTES + nv * BUILD_VERTEX_BYTES
        entry = {"ms": ms, "obs_points_per_s": obs.n / ms * 1e3,
                 "stage_ms": {"embed": st[0], "insert_and_ids": st[1], "values": st[2], "tables": st[3]},
                 "incidences": inc, "partial_records": part, "vertices": nv,
                 "algorithmic_bytes": alg, "table_bytes": nv * 2 * TABLE_SLOT_BYTES,
                 "achieved_gbs": alg / ms / 1e6,
                 "frac_of_hbm_peak": alg / ms / 1e6 / HBM_PEAK_GBS}
        if name == "sorted":
            entry["partial_record_bytes"] = part * PARTIAL_BYTES_SORTED
        else:
            atomics = part * ATOMICS_PER_PARTIAL
            scat = fr.fr_probe_atomics(ctx.h, 1 << 26, 1 << 30, True)
            pack = fr.fr_probe_atomics(ctx.h, 1 << 26, 1 << 30, False)
            rate = atomics / st[2] * 1e3
            entry["atomic_splat"] = {"atomics": atomics, "values_ms": st[2], "atomics_per_s": rate,
                                     "probe_scattered_atomics_per_s": scat, "probe_packed_atomics_per_s": pack,
                                     "frac_of_packed_probe": rate / pack,
                                     "note": "a wave's partial records carry vertex ids in first-touch order, so "
                                             "its atomics fall on few lines: between the scattered (one line "
                                             "per atomic) and packed (two lines per wave) probes"}
        res[name] = entry
    return res


def line_rates(fr, ctx):
    """The line-access ceiling of hash lookups: 16-byte lane loads, one lane per 128-byte line (a
    lookup's key or value read) and eight lanes per line, from an L2-resident (2 MiB) and an
    HBM-resident (1 GiB) table."""
    out = {}
    for where, nbytes in (("l2", 2 << 20), ("hbm", 1 << 30)):
        for g in (1, 8):
            out[f"{where}_lanes{g}_lines_per_s"] = fr.fr_probe_lines(ctx.h, g, nbytes)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--pairs", type=int, default=64)
    ap.add_argument("--iters", type=int, default=ITERS)
    ap.add_argument("--splat", choices=["sorted", "atomic"], default="sorted")
    ap.add_argument("--fused", type=int, default=1,
                    help="1: slice and reduction in one kernel (FR_FUSED, the default); 0: two kernels")
    ap.add_argument("--unfused-steps", type=int, default=3,
                    help="with --fused 1: steps of the two-kernel form timed after the headline, for comparison")
    ap.add_argument("--slice", choices=["auto", "plain", "shared"], default="auto",
                    help="E-step slice kernel (auto: the library's autotuner picks)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pairs", type=int, default=16, help="pairs the all-cores CPU oracle baseline runs")
    ap.add_argument("--copy-ref", action="store_true", help="end with plain copies of known size (counter scale)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--no-serve", action="store_true", help="skip the served request stream")
    ap.add_argument("--no-other", action="store_true", help="skip the single-pair workloads and build rates")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-slots", type=int, default=1024)
    ap.add_argument("--serve-arena", type=int, default=64 << 20)
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--serve-admit", type=int, default=32)
    ap.add_argument("--serve-tol", type=float, default=1e-6,
                    help="a request stops after a step with |omega| and |v| below this (0: all iterations)")
    ap.add_argument("--serve-capacity-requests", type=int, default=256)
    ap.add_argument("--serve-lambdas", type=float, nargs="*", default=[1.0, 2.0, 4.0, 8.0, 12.0, 16.0])
    ap.add_argument("--plain-lambdas", type=float, nargs="*", default=[1.0])
    ap.add_argument("--profile-workload", choices=["nodegraph", "articulated", "descriptors", "uncustomised",
                                                    "updated-sigma"],
                    help="run one single-pair workload a few times and exit (for kernel traces)")
    args = ap.parse_args()
    if args.profile_workload:
        profile_workload(args.profile_workload)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): independent pairs shard across GPUs "
              f"without communication, and the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    t = time.time()
    pairs = make_pairs(args.pairs, args.workers)
    M = [len(p.model) for p in pairs]
    N = [len(p.obs) for p in pairs]
    log(f"generated {len(pairs)} depth pairs in {time.time() - t:.1f} s: model {sum(M)} / obs {sum(N)} points")

    import torch
    import paper_1811_10136_amd as fr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    ctx = fr.Context(0)
    fr.fr_ctx_set_tuning(ctx.h, {"auto": fr.FR_SLICE_AUTO, "plain": fr.FR_SLICE_PLAIN,
                                 "shared": fr.FR_SLICE_SHARED}[args.slice])
    model = fr.Cloud.from_numpy([p.model for p in pairs], [p.model_n for p in pairs], dev)
    obs = fr.Cloud.from_numpy([p.obs for p in pairs], [p.obs_n for p in pairs], dev)
    sigma, sigma_n = pairs[0].sigma, pairs[0].sigma_n
    splat = fr.FR_SPLAT_SORTED if args.splat == "sorted" else fr.FR_SPLAT_ATOMIC
    prm = fr.register_params(6, "pt2pl", sigma, sigma_n, iters=args.iters, w=0.1, fixed=True, profile=True,
                             splat=splat, fused=bool(args.fused))
    T0 = np.repeat(np.eye(4)[None], len(pairs), 0)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        fr.register(ctx, model, obs, prm, T0=T0)
        log(f"warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    step_ms, est_ms, est_n, build_ms = [], 0.0, 0, []
    t_all = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        T, status, rep = fr.register(ctx, model, obs, prm, T0=T0)
        step_ms.append((time.perf_counter() - t0) * 1e3)
        est_ms += rep.estep_ms
        est_n += rep.estep_launches
        build_ms.append(rep.build_ms)
        log(f"step {i + 1}/{args.steps}: {step_ms[-1]:.2f} ms (build {rep.build_ms:.2f} ms, "
            f"E-step {rep.estep_ms / max(1, rep.estep_launches):.3f} ms/launch)")
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_all
    ms_per_step = total_s * 1e3 / args.steps

    # touched lattice vertices at the final poses (algorithmic table bytes of the E-step)
    lat = fr.Lattice(ctx, obs, prm.lattice)
    mats = torch.tensor(np.stack([Ti[:3, :4] for Ti in T]).astype(np.float32).reshape(-1), device=dev)
    xf = fr.XForm(fr.FR_XF_RIGID, mats, n_seg=len(pairs))
    touched = sum(fr.fr_estep_touched(lat.h, model, xf, s) for s in range(len(pairs)))
    n_vertices = sum(lat.stats(s)[0] for s in range(len(pairs)))
    lat.close()

    unfused = None
    if args.fused and args.unfused_steps > 0:
        # the same registrations with slice and reduction as two kernels, for comparison
        prm2 = fr.register_params(6, "pt2pl", sigma, sigma_n, iters=args.iters, w=0.1, fixed=True, profile=True,
                                  splat=splat, fused=False)
        fr.register(ctx, model, obs, prm2, T0=T0)   # warm-up (and the slice autotuner)
        torch.cuda.synchronize()
        u_est, u_n, u_m = 0.0, 0, 0.0
        t_u = time.perf_counter()
        for _ in range(args.unfused_steps):
            _, _, rep2 = fr.register(ctx, model, obs, prm2, T0=T0)
            u_est += rep2.estep_ms
            u_n += rep2.estep_launches
            u_m += rep2.mstep_ms
        torch.cuda.synchronize()
        u_s = (time.perf_counter() - t_u) / args.unfused_steps
        unfused = {"ms_per_step": u_s * 1e3, "value": sum(M) * args.iters / u_s,
                   "estep_ms_per_launch": u_est / max(1, u_n),
                   "reduction_ms_per_iter": u_m / (args.unfused_steps * args.iters),
                   "estep_roofline": {"bytes_per_point": EST_BYTES_PER_POINT,
                                      "achieved_gbs": (sum(M) * EST_BYTES_PER_POINT + touched * VERTEX_BYTES)
                                      / (u_est / max(1, u_n) / 1e3) / 1e9}}
        unfused["estep_roofline"]["frac"] = unfused["estep_roofline"]["achieved_gbs"] / HBM_PEAK_GBS
        log(f"two-kernel form: {unfused['ms_per_step']:.2f} ms/step, E-step {unfused['estep_ms_per_launch']:.3f} "
            f"ms/launch")

    points_per_launch = sum(M)
    per_point = FUSED_BYTES_PER_POINT if args.fused else EST_BYTES_PER_POINT
    tiles = sum((m + FUSED_TILE - 1) // FUSED_TILE for m in M)
    alg_bytes = points_per_launch * per_point + touched * VERTEX_BYTES + (tiles * PARTIAL_ROW_BYTES if args.fused else 0)
    est_avg_s = est_ms / max(1, est_n) / 1e3
    achieved = alg_bytes / est_avg_s / 1e9
    tuned = fr.fr_ctx_tuning_table(ctx.h)
    chosen = {"auto": None, "plain": fr.FR_SLICE_PLAIN, "shared": fr.FR_SLICE_SHARED}[args.slice]
    if chosen is None:
        kind = fr.FR_XF_RIGID + (TUNE_FUSED if args.fused else 0)
        big = [e for e in tuned if e["d"] == 6 and e["V"] == 7 and e["xf_kind"] == kind]
        chosen = max(big, key=lambda e: e["size_class"])["slice"] if big else fr.FR_SLICE_PLAIN
    if args.fused:
        kernel = "k_estep_fused<6,7,rigid,pt2pl,%s>" % fr.SLICE_NAMES[chosen]
    elif chosen == fr.FR_SLICE_SHARED:
        kernel = "k_estep_dedup<6,7,rigid>"
    else:
        kernel = "k_estep<6,7,rigid>"
    traffic = traffic_from_profile(points_per_launch, kernel)
    copy_gbs = copy_bandwidth()

    value = points_per_launch * args.iters * args.steps / total_s
    out = {
        "metric": "E-step points/sec (% HBM roofline); registrations/sec + p50/p99 latency",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batch of {len(pairs)} rigid point-to-plane depth-frame pairs (640x480 render of "
                        f"3 planes + 5 spheres, 2 mm noise, 5% dropout), d=6 features, {args.iters} EM iterations",
            "pairs": len(pairs), "model_points": points_per_launch, "obs_points": sum(N),
            "iters": args.iters, "sigma": sigma[0], "sigma_n": sigma_n, "splat": args.splat,
            "lattice_vertices": n_vertices, "touched_vertices": touched,
        },
        "registrations_per_s": len(pairs) * args.steps / total_s,
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "note": "latency of one batched step (all pairs of the batch complete together)"},
        "batch": {"registrations_per_s": len(pairs) * args.steps / total_s,
                  "step_ms_p50": float(np.percentile(step_ms, 50)), "step_ms_p99": float(np.percentile(step_ms, 99)),
                  "outcome": batch_outcome(pairs, T, status)},
        "build_ms_mean": float(np.mean(build_ms)),
        "autotuner": {"slice_mode": args.slice, "slice_used": fr.SLICE_NAMES[chosen], "table": tuned},
        "roofline": {
            "kernel": kernel,
            "bytes_per_point": per_point, "bytes_per_touched_vertex": VERTEX_BYTES,
            "partial_row_bytes_per_tile": PARTIAL_ROW_BYTES if args.fused else 0,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg_bytes,
            "mean_launch_ms": est_avg_s * 1e3,
            "measured_copy_gbs": copy_gbs,
            "frac_of_measured_copy": achieved / copy_gbs,
        },
    }
    if unfused is not None:
        out["unfused"] = unfused
    if not args.no_other:
        log("other workloads and build rates ...")
        out["other_workloads"] = other_workloads(fr, ctx)
        out["build"] = build_rates(fr, ctx, obs, sigma, sigma_n)
        out["roofline"]["line_rates"] = line_rates(fr, ctx)
    if not args.no_serve:
        out["serving"] = serve_bench(fr, ctx, args)
        h = out["serving"]["headline"]
        if h is not None:
            out["registrations_per_s"] = h["registrations_per_s"]
            out["latency_ms"] = {"p50": h["p50_ms"], "p99": h["p99_ms"],
                                 "note": f"served request stream at {h['lambda_x']}x the plain loop's capacity"}
            out["solved_per_s"] = h["solved_per_s"]
    if not args.no_cpu_baseline:
        log(f"timing the CPU oracle on {args.cpu_pairs} pairs ...")
        out["cpu_baseline"] = cpu_baseline(pairs[:args.cpu_pairs])
    if args.copy_ref:
        copy_reference()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
