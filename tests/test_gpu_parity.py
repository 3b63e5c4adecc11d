"""GPU parity: every call of the C ABI against the CPU oracle on the same seeded inputs.

Sizes span several tiles with ragged tails; tolerances are derived in _helpers.py.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from _helpers import (abs_scales, assert_estep_close, assert_lattice_equal, oracle_lattice, pose_close, soa,
                      upload, upper)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


RES = {4: "pt2pt", 7: "pt2pl"}
CASES = [(3, 4), (3, 7), (6, 4), (6, 7)]


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("splat", [0, 1], ids=["sorted", "atomic"])
@pytest.mark.parametrize("feat,V", CASES)
def test_lattice_build_parity(fr, ctx, feat, V, splat):
    p = synth.random_cloud_pair(21 + feat + V, 1000, 3001, feat=feat, residual=RES[V])
    _say(f"[lattice] feat={feat} V={V} splat={splat} N={len(p.obs)}")
    obs = upload([p.obs], [p.obs_n])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(feat, V, p.sigma, p.sigma_n, splat))
    keys, occ, vals = lat.export(0)
    ref = oracle_lattice(p.obs, p.obs_n, feat, RES[V], p.sigma, p.sigma_n)
    assert_lattice_equal(keys, occ, vals, ref, L=float(np.abs(p.obs).max()))
    nv, cap, _ = lat.stats(0)
    assert nv == ref.n_vertices and cap >= 2 * nv   # cuckoo load factor <= 0.5
    lat.close()


@pytest.mark.parametrize("splat", [0, 1], ids=["sorted", "atomic"])
def test_lattice_of_repeated_points(fr, ctx, splat):
    # 300 copies of one point among 500 others: whole tiles of splat records (256 each) carry the
    # same seven keys (the records of a tile are merged by key before they probe the global table),
    # and single vertices collect hundreds of incidences (few enough that the atomic mode's binary32
    # sums of equal terms stay within the vertex-value tolerance)
    p = synth.random_cloud_pair(7, 600, 500, feat=6, residual="pt2pl")
    obs = np.concatenate([p.obs[:200], np.repeat(p.obs[200:201], 300, 0), p.obs[201:]])
    obs_n = np.concatenate([p.obs_n[:200], np.repeat(p.obs_n[200:201], 300, 0), p.obs_n[201:]])
    _say(f"[lattice-repeat] splat={splat} N={len(obs)}")
    lat = fr.Lattice(ctx, upload([obs], [obs_n]), fr.lattice_params(6, 7, p.sigma, p.sigma_n, splat))
    keys, occ, vals = lat.export(0)
    ref = oracle_lattice(obs, obs_n, 6, "pt2pl", p.sigma, p.sigma_n)
    assert_lattice_equal(keys, occ, vals, ref, L=float(np.abs(obs).max()))
    assert occ.max() >= 300
    M = len(p.model)
    m0, m1 = torch.empty(M, device="cuda"), torch.empty(3 * M, device="cuda")
    ns = torch.empty(3 * M, device="cuda")
    model = upload([p.model], [p.model_n])
    fr.fr_estep(lat.h, model, fr.XForm(), m0, m1, ns)
    torch.cuda.synchronize()
    g = oracle.lattice_slice(ref, oracle.features(p.model, p.model_n, 6))
    assert_estep_close(soa(m0), soa(m1).reshape(3, M).T, soa(ns).reshape(3, M).T, g[:, 0], g[:, 1:4], g[:, 4:7],
                       float(ref.vals[:, 0].max()), float(np.abs(obs).max()))
    lat.close()


def test_provisional_table_overflow_and_sizing_from_the_previous_build(fr):
    # points farther apart than the kernel: every splat record carries a key of its own, so a fresh
    # context's first provisional table (sized for half the records) overflows and the insertion runs
    # again in a larger one; the next build in that context sizes its table from this one's vertices
    # per record and inserts once.  Both give the oracle's lattice.
    p = synth.separated_pair(3, m=3000, sigma=0.02, feat=6, residual="pt2pl")
    _say(f"[provisional] N={len(p.obs)}")
    c = fr.Context(0)
    ref = oracle_lattice(p.obs, p.obs_n, 6, "pt2pl", p.sigma, p.sigma_n)
    assert ref.n_vertices > 0.5 * 7 * len(p.obs)          # more keys than the first table takes
    outs = []
    for _ in range(2):
        lat = fr.Lattice(c, upload([p.obs], [p.obs_n]), fr.lattice_params(6, 7, p.sigma, p.sigma_n))
        keys, occ, vals = lat.export(0)
        assert_lattice_equal(keys, occ, vals, ref, L=float(np.abs(p.obs).max()))
        outs.append((keys, occ, vals))
        lat.close()
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)
    c.close()


@pytest.mark.parametrize("splat", [0, 1], ids=["sorted", "atomic"])
def test_lattice_full_depth_frame(fr, ctx, splat):
    p = synth.depth_pair(0)
    _say(f"[lattice-full] depth frame N={len(p.obs)} d=6 V=7 splat={splat}")
    obs = upload([p.obs], [p.obs_n])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(6, 7, p.sigma, p.sigma_n, splat))
    keys, occ, vals = lat.export(0)
    ref = oracle_lattice(p.obs, p.obs_n, 6, "pt2pl", p.sigma, p.sigma_n)
    assert_lattice_equal(keys, occ, vals, ref, L=float(np.abs(p.obs).max()))
    assert occ.sum() == 7 * len(p.obs)
    lat.close()


def _estep_case(fr, ctx, p, feat, V, T):
    res = RES[V]
    obs = upload([p.obs], [p.obs_n])
    model = upload([p.model], [p.model_n])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(feat, V, p.sigma, p.sigma_n, 0))
    M = len(p.model)
    mat = oracle.pose_to_mat12(T)
    mats = torch.from_numpy(mat.copy()).cuda()
    xf = fr.XForm(fr.FR_XF_RIGID, mats, n_seg=1)
    m0 = torch.empty(M, device="cuda")
    m1 = torch.empty(3 * M, device="cuda")
    ns = torch.empty(3 * M, device="cuda") if V == 7 else None
    fr.fr_estep(lat.h, model, xf, m0, m1, ns)
    torch.cuda.synchronize()
    ref_lat = oracle_lattice(p.obs, p.obs_n, feat, res, p.sigma, p.sigma_n)
    x32 = oracle.transform_f32(mat, p.model)
    n32 = oracle.transform_f32(mat, p.model_n, translate=False)
    g, touched = oracle.lattice_slice(ref_lat, oracle.features(x32, n32, feat), return_touched=True)
    vmax = float(ref_lat.vals[:, 0].max())
    assert_estep_close(soa(m0), soa(m1).reshape(3, M).T, soa(ns).reshape(3, M).T if ns is not None else None,
                       g[:, 0], g[:, 1:4], g[:, 4:7] if V == 7 else None, vmax, float(np.abs(p.obs).max()))
    return lat, model, xf, touched, g


@pytest.mark.parametrize("feat,V", CASES)
def test_estep_parity(fr, ctx, feat, V):
    p = synth.random_cloud_pair(31 + feat + V, 2777, 2500, feat=feat, residual=RES[V])
    _say(f"[estep] feat={feat} V={V} M={len(p.model)}")
    T = synth.random_motion(np.random.default_rng(feat * V), math.radians(2.0), 0.005)
    lat, model, xf, touched, g = _estep_case(fr, ctx, p, feat, V, T)
    assert (g[:, 0] > 0).mean() > 0.5
    assert fr.fr_estep_touched(lat.h, model, xf, 0) == touched
    lat.close()


def test_estep_identity_xform_and_segments(fr, ctx):
    """FR_XF_NONE equals FR_XF_RIGID with the identity; a segmented transform equals per-segment rigid."""
    p = synth.random_cloud_pair(77, 1500, 1500, feat=3, residual="pt2pt")
    obs = upload([p.obs])
    model = upload([p.model])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(3, 4, p.sigma))
    M = len(p.model)
    outs = []
    eye = torch.tensor(np.eye(4)[:3].reshape(12), dtype=torch.float32, device="cuda")
    for kind, mats in ((fr.FR_XF_NONE, None), (fr.FR_XF_RIGID, eye)):
        xf = fr.XForm(kind, mats, n_seg=1 if mats is not None else 0)
        m0 = torch.empty(M, device="cuda")
        m1 = torch.empty(3 * M, device="cuda")
        fr.fr_estep(lat.h, model, xf, m0, m1)
        outs.append((soa(m0), soa(m1)))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    # three segments with different motions
    rng = np.random.default_rng(5)
    Ts = [synth.random_motion(rng, 0.03, 0.004) for _ in range(3)]
    off = [0, 400, 401, M]
    mats = torch.from_numpy(np.concatenate([oracle.pose_to_mat12(T) for T in Ts])).cuda()
    xf = fr.XForm(fr.FR_XF_SEGMENTED, mats, seg_offsets=off)
    m0 = torch.empty(M, device="cuda")
    m1 = torch.empty(3 * M, device="cuda")
    fr.fr_estep(lat.h, model, xf, m0, m1)
    ref_lat = oracle_lattice(p.obs, None, 3, "pt2pt", p.sigma, p.sigma_n)
    x32 = np.concatenate([oracle.transform_f32(oracle.pose_to_mat12(Ts[s]), p.model[off[s]:off[s + 1]])
                          for s in range(3)])
    g = oracle.lattice_slice(ref_lat, oracle.features(x32, None, 3))
    assert_estep_close(soa(m0), soa(m1).reshape(3, M).T, None, g[:, 0], g[:, 1:4], None,
                       float(ref_lat.vals[:, 0].max()), float(np.abs(p.obs).max()))
    lat.close()


def test_estep_full_size_depth_frame_sampled(fr, ctx):
    """Config-2 scale (about 260k points, d = 6, V = 7) in the launch configuration of the benchmark;
    the oracle checks a sample of 4000 points one by one."""
    p = synth.depth_pair(2)
    _say(f"[estep-full] M={len(p.model)} N={len(p.obs)}")
    obs = upload([p.obs], [p.obs_n])
    model = upload([p.model], [p.model_n])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(6, 7, p.sigma, p.sigma_n, 0))
    M = len(p.model)
    T = p.T_gt @ oracle.se3_exp(np.array([0.003, -0.002, 0.001, 0.004, 0.002, -0.003]))
    mat = oracle.pose_to_mat12(T)
    xf = fr.XForm(fr.FR_XF_RIGID, torch.from_numpy(mat.copy()).cuda(), n_seg=1)
    m0 = torch.empty(M, device="cuda")
    m1 = torch.empty(3 * M, device="cuda")
    ns = torch.empty(3 * M, device="cuda")
    fr.fr_estep(lat.h, model, xf, m0, m1, ns)
    idx = np.sort(np.random.default_rng(0).choice(M, 4000, replace=False))
    ref_lat = oracle_lattice(p.obs, p.obs_n, 6, "pt2pl", p.sigma, p.sigma_n)
    x32 = oracle.transform_f32(mat, p.model[idx])
    n32 = oracle.transform_f32(mat, p.model_n[idx], translate=False)
    g = oracle.lattice_slice(ref_lat, oracle.features(x32, n32, 6))
    assert (g[:, 0] > 0).mean() > 0.5
    assert_estep_close(soa(m0)[idx], soa(m1).reshape(3, M).T[idx], soa(ns).reshape(3, M).T[idx], g[:, 0],
                       g[:, 1:4], g[:, 4:7], float(ref_lat.vals[:, 0].max()), float(np.abs(p.obs).max()))
    # property at any size: M0 >= 0 everywhere and M1/M0 within the lattice's bounding box
    a0 = soa(m0)
    assert a0.min() >= 0.0
    lat.close()


@pytest.mark.parametrize("residual", ["pt2pt", "pt2pl"])
def test_mstep_reduce_parity(fr, ctx, residual):
    rng = np.random.default_rng(3)
    M = 5000 + 333
    x_ref = rng.normal(scale=0.5, size=(M, 3)).astype(np.float32)
    m0 = rng.uniform(0.0, 3.0, size=M).astype(np.float32)
    m0[rng.uniform(size=M) < 0.2] = 0.0
    m1 = ((x_ref + rng.normal(scale=0.01, size=(M, 3))) * m0[:, None]).astype(np.float32)
    ns = (rng.normal(size=(M, 3)) * m0[:, None]).astype(np.float32)
    T = synth.random_motion(rng, 0.2, 0.1)
    mat = oracle.pose_to_mat12(T)
    model = upload([x_ref])
    xf = fr.XForm(fr.FR_XF_RIGID, torch.from_numpy(mat.copy()).cuda(), n_seg=1)
    tm0 = torch.from_numpy(m0).cuda()
    tm1 = torch.from_numpy(np.ascontiguousarray(m1.T).reshape(-1)).cuda()
    tns = torch.from_numpy(np.ascontiguousarray(ns.T).reshape(-1)).cuda()
    jtj = torch.zeros(21, dtype=torch.float64, device="cuda")
    jtr = torch.zeros(6, dtype=torch.float64, device="cuda")
    st = torch.zeros(4, dtype=torch.float64, device="cuda")
    c, sigma = 0.37, 0.02
    res = fr.FR_PT2PL if residual == "pt2pl" else fr.FR_PT2PT
    fr.fr_mstep_reduce(model, xf, tm0, tm1, tns, res, c, sigma, jtj, jtr, st)
    R = mat.reshape(3, 4).astype(np.float64)
    x64 = x_ref.astype(np.float64) @ R[:, :3].T + R[:, 3]
    A, b, stats = oracle.normal_equations(x64, m0, m1, ns, c, sigma, residual)
    sA, sb = abs_scales(x64, m0, m1, ns, c, sigma, residual)
    assert (np.abs(soa(jtj) - upper(A)) <= 1e-5 * upper(sA) + 1e-12).all()
    assert (np.abs(soa(jtr) - b) <= 1e-5 * sb + 1e-12).all()
    np.testing.assert_allclose(soa(st), stats, rtol=1e-5)


def test_mstep_reduce_segments_and_bitwise_repeat(fr, ctx):
    rng = np.random.default_rng(9)
    M = 4099
    x_ref = rng.normal(size=(M, 3)).astype(np.float32)
    m0 = rng.uniform(0.1, 2.0, size=M).astype(np.float32)
    m1 = (x_ref * m0[:, None]).astype(np.float32) + 0.01
    off = [0, 1000, 1000, 3100, M]
    Ts = [synth.random_motion(rng, 0.1, 0.05) for _ in range(4)]
    mats = torch.from_numpy(np.concatenate([oracle.pose_to_mat12(T) for T in Ts])).cuda()
    model = upload([x_ref])
    xf = fr.XForm(fr.FR_XF_SEGMENTED, mats, seg_offsets=off)
    tm0 = torch.from_numpy(m0).cuda()
    tm1 = torch.from_numpy(np.ascontiguousarray(m1.T).reshape(-1)).cuda()
    outs = []
    for _ in range(2):
        jtj = torch.zeros(4 * 21, dtype=torch.float64, device="cuda")
        jtr = torch.zeros(4 * 6, dtype=torch.float64, device="cuda")
        st = torch.zeros(4 * 4, dtype=torch.float64, device="cuda")
        fr.fr_mstep_reduce(model, xf, tm0, tm1, None, fr.FR_PT2PT, 0.5, 0.03, jtj, jtr, st)
        outs.append((soa(jtj), soa(jtr), soa(st)))
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)
    for s in range(4):
        sl = slice(off[s], off[s + 1])
        R = oracle.pose_to_mat12(Ts[s]).reshape(3, 4).astype(np.float64)
        x64 = x_ref[sl].astype(np.float64) @ R[:, :3].T + R[:, 3]
        A, b, stats = oracle.normal_equations(x64, m0[sl], m1[sl], None, 0.5, 0.03, "pt2pt")
        sA, sb = abs_scales(x64, m0[sl], m1[sl], None, 0.5, 0.03, "pt2pt")
        assert (np.abs(outs[0][0][21 * s:21 * s + 21] - upper(A)) <= 1e-5 * upper(sA) + 1e-12).all()
        assert (np.abs(outs[0][1][6 * s:6 * s + 6] - b) <= 1e-5 * sb + 1e-12).all()
        np.testing.assert_allclose(outs[0][2][4 * s:4 * s + 4], stats, rtol=1e-5, atol=1e-12)


def test_solve_rigid_parity(fr, ctx):
    rng = np.random.default_rng(4)
    n = 7
    As, bs, Ts = [], [], []
    for i in range(n):
        G = rng.normal(size=(6, 6))
        As.append(G @ G.T + 0.1 * np.eye(6))
        bs.append(rng.normal(size=6) * 10 ** rng.uniform(-6, -1))
        Ts.append(synth.random_motion(rng, 1.0, 1.0))
    As[3] = np.zeros((6, 6))   # degenerate
    jtj = torch.tensor(np.concatenate([upper(A) for A in As]), dtype=torch.float64, device="cuda")
    jtr = torch.tensor(np.concatenate(bs), dtype=torch.float64, device="cuda")
    poses = torch.tensor(np.stack(Ts).reshape(-1), dtype=torch.float64, device="cuda")
    mats = torch.zeros(n * 12, dtype=torch.float32, device="cuda")
    tn = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    status = torch.zeros(n, dtype=torch.int32, device="cuda")
    fr.fr_solve_rigid(n, jtj, jtr, poses, mats, tn, status)
    P = soa(poses).reshape(n, 4, 4)
    S = soa(status)
    for i in range(n):
        if i == 3:
            assert S[i] == fr.FR_EDEGENERATE
            np.testing.assert_array_equal(P[i], Ts[i])
            continue
        assert S[i] == 0
        dz = oracle.gn_step(As[i], bs[i])
        ref = oracle.se3_exp(dz) @ Ts[i]
        np.testing.assert_allclose(P[i], ref, atol=1e-12)
        np.testing.assert_array_equal(soa(mats).reshape(n, 12)[i], oracle.pose_to_mat12(ref))
        np.testing.assert_allclose(soa(tn).reshape(n, 2)[i], [np.linalg.norm(dz[:3]), np.linalg.norm(dz[3:])],
                                   rtol=1e-12)


def test_register_parity_ellipsoid(fr, ctx):
    p = synth.ellipsoid_pair(1)
    _say(f"[register] ellipsoid M={len(p.model)} N={len(p.obs)} pt2pt d=3, 30 iterations")
    T0 = p.T_gt @ oracle.se3_exp(np.array([0.01, -0.01, 0.005, 0.004, 0.0, -0.003]))
    ref = oracle.register_rigid(p.model, None, p.obs, None, feat=3, residual="pt2pt", sigma=p.sigma, w=p.w,
                                iters=p.iters, T0=T0)
    prm = fr.register_params(3, "pt2pt", p.sigma, iters=p.iters, w=p.w)
    T, status, rep = fr.register(ctx, upload([p.model]), upload([p.obs]), prm, T0=T0[None])
    ang, dt, ok = pose_close(T[0], ref)
    assert status[0] == 0 and ok, (ang, dt)
    assert rep.iterations == p.iters


@pytest.mark.parametrize("feat,residual", [(3, "pt2pt"), (6, "pt2pl"), (3, "pt2pl")])
def test_register_exact_recovery(fr, ctx, feat, residual):
    p = synth.separated_pair(8, 700, feat=feat, residual=residual)
    prm = fr.register_params(feat, residual, p.sigma, p.sigma_n, iters=12, c=0.0)
    T, status, _ = fr.register(ctx, upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n]), prm,
                               T0=p.extra["T0"][None])
    assert status[0] == 0
    assert np.abs(T[0] - p.T_gt).max() < 1e-5
    assert oracle.alignment_error(T[0], p.T_gt, p.model) < 1e-5


@pytest.mark.parametrize("fused", [False, True])
def test_register_parity_depth_batch_and_alone_bitwise(fr, ctx, fused):
    """Three depth pairs of different sizes registered alone and as one batch: identical poses,
    all within tolerance of the oracle (also with the slice and the reduction fused)."""
    pairs = [synth.depth_pair(s, width=w, height=h, f=f) for s, (w, h, f) in
             enumerate([(160, 120, 131.25), (96, 72, 78.75), (200, 150, 164.06)])]
    T0s = [q.T_gt @ oracle.se3_exp(np.array([0.004, -0.003, 0.002, 0.004, 0.003, -0.002])) for q in pairs]
    prm = fr.register_params(6, "pt2pl", pairs[0].sigma, pairs[0].sigma_n, iters=15, w=0.1, fused=fused)
    _say(f"[register] depth batch of 3 {[len(q.model) for q in pairs]} fused={fused}")
    Tb, sb, _ = fr.register(ctx, upload([q.model for q in pairs], [q.model_n for q in pairs]),
                            upload([q.obs for q in pairs], [q.obs_n for q in pairs]), prm, T0=np.stack(T0s))
    assert (sb == 0).all()
    for i, q in enumerate(pairs):
        Ta, sa, _ = fr.register(ctx, upload([q.model], [q.model_n]), upload([q.obs], [q.obs_n]), prm,
                                T0=T0s[i][None])
        np.testing.assert_array_equal(Ta[0], Tb[i])
        ref = oracle.register_rigid(q.model, q.model_n, q.obs, q.obs_n, feat=6, residual="pt2pl", sigma=q.sigma,
                                    sigma_n=q.sigma_n, w=0.1, iters=15, T0=T0s[i])
        ang, dt, ok = pose_close(Tb[i], ref)
        assert ok, (i, ang, dt)


def test_sorted_build_is_bitwise_deterministic(fr, ctx):
    p = synth.depth_pair(5, width=320, height=240, f=262.5)
    obs = upload([p.obs], [p.obs_n])
    a = fr.Lattice(ctx, obs, fr.lattice_params(6, 7, p.sigma, p.sigma_n, 0)).export(0)
    b = fr.Lattice(ctx, obs, fr.lattice_params(6, 7, p.sigma, p.sigma_n, 0)).export(0)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    c = fr.Lattice(ctx, obs, fr.lattice_params(6, 7, p.sigma, p.sigma_n, 1)).export(0)
    np.testing.assert_array_equal(a[0], c[0])
    np.testing.assert_array_equal(a[1], c[1])
    np.testing.assert_allclose(a[2], c[2], rtol=1e-5, atol=1e-5)


def test_edge_cases(fr, ctx):
    p = synth.random_cloud_pair(2, 300, 301)
    # a batch with an empty observation set, an empty model set and a single point
    obs = upload([p.obs, np.zeros((0, 3), np.float32), p.obs[:1], p.obs[:50]])
    model = upload([p.model, p.model[:10], np.zeros((0, 3), np.float32), p.model[:50]])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(3, 4, p.sigma))
    assert lat.stats(1)[0] == 0 and lat.stats(2)[0] == 4
    M = model.n
    m0 = torch.full((M,), -1.0, device="cuda")
    m1 = torch.full((3 * M,), -1.0, device="cuda")
    xf = fr.XForm(fr.FR_XF_NONE)
    fr.fr_estep(lat.h, model, xf, m0, m1)
    a0 = soa(m0)
    assert (a0[300:310] == 0).all()          # empty lattice -> no support, zeros written
    for s, (o, y) in enumerate([(p.obs, p.model), (None, None), (p.obs[:1], None), (p.obs[:50], p.model[:50])]):
        if y is None:
            continue
        ref = oracle_lattice(o, None, 3, "pt2pt", p.sigma, 0.5)
        g = oracle.lattice_slice(ref, oracle.features(y, None, 3))
        lo = int(model.offsets[s])
        np.testing.assert_allclose(a0[lo:lo + len(y)], g[:, 0], rtol=1e-5, atol=1e-6)
    lat.close()
    # registration of a pair with no observation is degenerate, the others still succeed
    prm = fr.register_params(3, "pt2pt", p.sigma, iters=3, w=0.0)
    T, status, _ = fr.register(ctx, upload([p.model, p.model]), upload([p.obs, np.zeros((0, 3), np.float32)]), prm)
    assert status[0] == 0 and status[1] == fr.FR_EDEGENERATE
    # key range overflow is reported, not silently wrapped
    far = (p.obs * 0 + 1.0e5).astype(np.float32)
    with pytest.raises(fr.FRError) as e:
        fr.Lattice(ctx, upload([far]), fr.lattice_params(3, 4, (0.01, 0.01, 0.01)))
    assert e.value.status == fr.FR_ERANGE
    # argument errors
    with pytest.raises(fr.FRError) as e:
        fr.Lattice(ctx, upload([p.obs]), fr.lattice_params(3, 4, (0.0, 0.01, 0.01)))
    assert e.value.status == fr.FR_EINVAL
    with pytest.raises(fr.FRError) as e:
        fr.Lattice(ctx, upload([p.obs]), fr.lattice_params(6, 7, p.sigma))   # feat 6 without normals
    assert e.value.status == fr.FR_EINVAL


def test_budget_is_enforced(fr):
    p = synth.random_cloud_pair(2, 300, 3000)
    small = fr.Context(0, hbm_budget_bytes=64 * 1024)
    with pytest.raises(fr.FRError) as e:
        fr.Lattice(small, upload([p.obs]), fr.lattice_params(3, 4, p.sigma))
    assert e.value.status == fr.FR_EBUDGET
    assert fr.fr_ctx_usage(small.h) == 0
    small.close()


@pytest.mark.parametrize("feat,residual", [(3, "pt2pt"), (3, "pt2pl"), (6, "pt2pt")])
def test_register_fused_matches_oracle_other_variants(fr, ctx, feat, residual):
    """The fused slice + reduction for the other feature/residual combinations, from a start near
    the ground truth, against the oracle."""
    q = synth.depth_pair(9, width=160, height=120, f=131.25)
    T0 = q.T_gt @ oracle.se3_exp(np.array([0.003, 0.002, -0.003, -0.003, 0.002, 0.003]))
    prm = fr.register_params(feat, residual, q.sigma, q.sigma_n, iters=10, w=0.1, fused=True)
    nrm = feat == 6 or residual == "pt2pl"
    T, st, _ = fr.register(ctx, upload([q.model], [q.model_n] if feat == 6 else None),
                           upload([q.obs], [q.obs_n] if nrm else None), prm, T0=T0[None])
    ref = oracle.register_rigid(q.model, q.model_n if feat == 6 else None, q.obs, q.obs_n if nrm else None,
                                feat=feat, residual=residual, sigma=q.sigma, sigma_n=q.sigma_n, w=0.1, iters=10,
                                T0=T0)
    assert int(st[0]) == 0
    ang, dt, ok = pose_close(T[0], ref)
    assert ok, (ang, dt)


@pytest.mark.parametrize("feat,residual", [(6, "pt2pl"), (3, "pt2pt")])
def test_fused_shared_and_plain_slices_agree_bitwise(fr, ctx, feat, residual):
    """The fused slice + reduction with the shared-lookup slice and with the per-point slice: their slice
    sums are bitwise the same and the reduction is one code, so the poses must be identical; both are
    held to the oracle."""
    q = synth.depth_pair(4, width=320, height=240, f=262.5)
    T0 = q.T_gt @ oracle.se3_exp(np.array([0.004, -0.003, 0.002, 0.004, 0.003, -0.002]))
    prm = fr.register_params(feat, residual, q.sigma, q.sigma_n, iters=12, w=0.1, fused=True)
    nrm = feat == 6 or residual == "pt2pl"
    model = upload([q.model], [q.model_n] if feat == 6 else None)
    obs = upload([q.obs], [q.obs_n] if nrm else None)
    _say(f"[fused-forms] feat={feat} {residual} model {len(q.model)} points")
    T = {}
    try:
        for sl in (fr.FR_SLICE_PLAIN, fr.FR_SLICE_SHARED):
            fr.fr_ctx_set_tuning(ctx.h, sl)
            T[sl], st, _ = fr.register(ctx, model, obs, prm, T0=T0[None])
            assert int(st[0]) == 0
    finally:
        fr.fr_ctx_set_tuning(ctx.h, fr.FR_SLICE_AUTO)
    np.testing.assert_array_equal(T[fr.FR_SLICE_PLAIN], T[fr.FR_SLICE_SHARED])
    ref = oracle.register_rigid(q.model, q.model_n if feat == 6 else None, q.obs, q.obs_n if nrm else None,
                                feat=feat, residual=residual, sigma=q.sigma, sigma_n=q.sigma_n, w=0.1, iters=12,
                                T0=T0)
    ang, dt, ok = pose_close(T[fr.FR_SLICE_SHARED][0], ref)
    assert ok, (ang, dt)


@pytest.mark.parametrize("feat,residual", [(6, "pt2pl"), (3, "pt2pt")])
def test_fused_points_without_support_add_nothing(fr, ctx, feat, residual):
    """Eq. 7 / Eq. 10 weigh a model point by M0 / (M0 + c): a point whose simplex meets no lattice vertex
    (M0 = 0) has weight 0, and the fused step adds exact zeros for it whatever its position and normal.
    Appending 300 model points 10 m away from the frame (they fill the lanes past the cloud's end and a
    tile of their own) must leave every pose bitwise unchanged, with either slice form.  c is given
    explicitly, since its rule scales with the number of model points."""
    q = synth.depth_pair(7, width=160, height=120, f=131.25)
    sig = np.broadcast_to(np.asarray(q.sigma, dtype=np.float64), (3,))
    c = oracle.outlier_constant(0.1, len(q.obs), len(q.model), oracle.feature_sigmas(feat, sig, q.sigma_n))
    prm = fr.register_params(feat, residual, q.sigma, q.sigma_n, iters=8, w=0.1, c=c, fused=True)
    nrm = feat == 6 or residual == "pt2pl"
    far = (q.model[:300] + np.array([10.0, -10.0, 10.0], dtype=np.float32)).astype(np.float32)
    clouds = {
        "alone": upload([q.model], [q.model_n] if feat == 6 else None),
        "with far points": upload([np.concatenate([q.model, far])],
                                  [np.concatenate([q.model_n, q.model_n[:300]])] if feat == 6 else None),
    }
    obs = upload([q.obs], [q.obs_n] if nrm else None)
    T0 = q.T_gt @ oracle.se3_exp(np.array([0.004, -0.003, 0.002, 0.004, 0.003, -0.002]))
    _say(f"[fused-far] feat={feat} {residual} model {len(q.model)} + 300 far points")
    try:
        for sl in (fr.FR_SLICE_PLAIN, fr.FR_SLICE_SHARED):
            fr.fr_ctx_set_tuning(ctx.h, sl)
            res = {k: fr.register(ctx, m, obs, prm, T0=T0[None]) for k, m in clouds.items()}
            assert int(res["alone"][1][0]) == 0
            np.testing.assert_array_equal(res["alone"][0], res["with far points"][0])
            np.testing.assert_array_equal(res["alone"][1], res["with far points"][1])
    finally:
        fr.fr_ctx_set_tuning(ctx.h, fr.FR_SLICE_AUTO)


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("fixed", [True, False])
def test_graph_replay_equals_the_eager_loop(fr, ctx, fixed, fused):
    """With FR_GRAPH, fr_register replays its iterations from a captured HIP graph (FR_PROFILE_EVENTS
    launches every kernel eagerly).  Several calls, each replaying its graph
    (several times in the early-stopping mode, with the host's checks between replays), give the eager
    loop's poses, statuses and iteration counts bitwise."""
    pairs = [synth.depth_pair(40 + i, width=w, height=h, f=f)
             for i, (w, h, f) in enumerate([(160, 120, 131.25), (96, 72, 78.75), (200, 150, 164.0)])]
    q = pairs[0]
    _say(f"[graph] fixed={fixed} fused={fused} sizes={[len(p.model) for p in pairs]}")
    model = upload([p.model for p in pairs], [p.model_n for p in pairs])
    obs = upload([p.obs for p in pairs], [p.obs_n for p in pairs])
    T0 = np.stack([p.T_gt @ oracle.se3_exp(np.array([0.01, -0.01, 0.005, 0.01, 0.005, -0.01])) for p in pairs])
    kw = dict(iters=14, w=q.w, fixed=fixed, fused=fused, tol=1e-5)
    eager = fr.register(ctx, model, obs, fr.register_params(6, "pt2pl", q.sigma, q.sigma_n, profile=True, **kw),
                        T0=T0)
    for _ in range(3):
        T, st, rep = fr.register(ctx, model, obs, fr.register_params(6, "pt2pl", q.sigma, q.sigma_n, graph=True,
                                                                     **kw), T0=T0)
        np.testing.assert_array_equal(T, eager[0])
        np.testing.assert_array_equal(st, eager[1])
        assert rep.iterations == eager[2].iterations
    if not fixed:
        assert eager[2].iterations < 14     # stopped early: the graph was replayed several times


def test_graph_blocks_and_remainder_equal_the_eager_loop(fr, ctx):
    """40 fixed iterations: one 32-iteration graph replay, then 8 iterations launched eagerly."""
    p = synth.ellipsoid_pair(6)
    _say("[graph] 40 fixed iterations")
    m, o = upload([p.model]), upload([p.obs])
    kw = dict(iters=40, w=p.w, fixed=True)
    eager = fr.register(ctx, m, o, fr.register_params(3, "pt2pt", p.sigma, profile=True, **kw))
    for _ in range(2):
        T, st, rep = fr.register(ctx, m, o, fr.register_params(3, "pt2pt", p.sigma, graph=True, **kw))
        np.testing.assert_array_equal(T, eager[0])
        assert rep.iterations == 40 and st[0] == eager[1][0]


def _twist_sizes(hist):
    return [max(np.linalg.norm(h["dz"][:3]), np.linalg.norm(h["dz"][3:])) for h in hist]


@pytest.mark.parametrize("case", ["ellipsoid", "depth", "depth_far"])
def test_stop_on_twist_matches_the_oracle_stop_iteration(fr, ctx, case):
    """Iteration control (Sec. 6.1): without FR_FIXED_ITERS the device stops a set after the first step
    whose rotation and translation parts both fall below twist_tol; the oracle applies the same rule.
    Stop iterations must agree, except where the oracle's decisive twist lies within 25% of the
    tolerance (binary32 sums move a twist by about 1e-6 of its size, so only a near tie may split)."""
    tol = 1e-5
    if case == "ellipsoid":
        p = synth.ellipsoid_pair(3)
        T0 = p.T_gt @ oracle.se3_exp(np.array([0.02, -0.01, 0.01, 0.005, 0.004, -0.003]))
        kw = dict(feat=3, residual="pt2pt")
    else:
        p = synth.depth_pair(7 if case == "depth" else 8, width=160, height=120, f=131.25)
        d = 0.004 if case == "depth" else 0.012
        T0 = p.T_gt @ oracle.se3_exp(np.array([d, -d, d / 2, d, d / 2, -d]))
        kw = dict(feat=6, residual="pt2pl")
    _say(f"[stop] {case} M={len(p.model)} tol={tol}")
    hist, info = [], {}
    ref = oracle.register_rigid(p.model, p.model_n, p.obs, p.obs_n, sigma=p.sigma, sigma_n=p.sigma_n, w=p.w,
                                iters=60, T0=T0, twist_tol=tol, history=hist, info=info, **kw)
    prm = fr.register_params(kw["feat"], kw["residual"], p.sigma, p.sigma_n, iters=60, w=p.w, fixed=False, tol=tol)
    T, st, rep = fr.register(ctx, upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n]), prm, T0=T0[None])
    assert st[0] == 0
    k = info["iterations"]
    assert 2 <= k < 60, k
    tw = _twist_sizes(hist)
    clear = tw[k - 1] < 0.75 * tol and tw[k - 2] > 1.25 * tol
    if clear:
        assert rep.iterations == k, (rep.iterations, k, tw[k - 3:k])
    else:
        assert abs(rep.iterations - k) <= 1, (rep.iterations, k, tw[k - 3:k])
    ang, dt, ok = pose_close(T[0], ref)
    assert ok, (ang, dt)


def test_stop_on_twist_batch_equals_each_pair_alone(fr, ctx):
    """Sets of one call stop at different iterations on the device; each ends bitwise where it ends
    alone, and the call reports the largest count."""
    pairs = [synth.depth_pair(60 + i, width=w, height=h, f=f)
             for i, (w, h, f) in enumerate([(160, 120, 131.25), (96, 72, 78.75), (200, 150, 164.0)])]
    T0 = np.stack([p.T_gt @ oracle.se3_exp(np.array([0.003 * (i + 1), -0.004, 0.002, 0.01 * (i + 1), 0.0, -0.005]))
                   for i, p in enumerate(pairs)])
    q = pairs[0]
    prm = fr.register_params(6, "pt2pl", q.sigma, q.sigma_n, iters=50, w=q.w, fixed=False, tol=1e-5)
    T, st, rep = fr.register(ctx, upload([p.model for p in pairs], [p.model_n for p in pairs]),
                             upload([p.obs for p in pairs], [p.obs_n for p in pairs]), prm, T0=T0)
    its = []
    for i, p in enumerate(pairs):
        Ta, sa, ra = fr.register(ctx, upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n]), prm,
                                 T0=T0[i][None])
        np.testing.assert_array_equal(T[i], Ta[0])
        assert st[i] == sa[0]
        its.append(ra.iterations)
    assert rep.iterations == max(its) and len(set(its)) > 1, its
