"""GPU parity of the uncustomised filter: the joint lattice of [Y, X], its blur, the slice, and the EM
loop that rebuilds and blurs the lattice every iteration (FR_BLURRED), against the oracle.

Tolerances: keys and occupancy bit-exact; splat values as _helpers.py; blurred values are convex
combinations (weights 1/4, 1/2) of splat values, so they keep the splat tolerance taken against the
largest value of the set; slices as _helpers.py.  EM: one step from the oracle's state matches to the
usual pose tolerance; many steps are held to 1e-3, because a model point that moves across a cell
boundary adds or removes a zero-valued vertex through which the blur passes.
"""
import numpy as np
import pytest

import oracle
import synth
from _helpers import assert_estep_close, pose_close, soa, upload

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


def _say(msg):
    print(msg, flush=True)


RES = {4: "pt2pt", 7: "pt2pl"}
CASES = [(3, 4), (3, 7), (6, 4), (6, 7)]


def _close_vals(vals, ref, L, what):
    vmax = float(np.abs(ref[:, 0]).max())
    scale = np.maximum(1.0, np.abs(ref[:, :1]))
    colL = np.ones(ref.shape[1])
    colL[1:4] = L
    tol = 1e-5 * scale * colL[None, :] + 1e-6 * vmax * colL[None, :]
    err = np.abs(vals.astype(np.float64) - ref)
    assert (err <= tol).all(), f"{what}: {(err > tol).sum()} values off; worst {err.max():.3e}"


@pytest.mark.parametrize("splat", [0, 1], ids=["sorted", "atomic"])
@pytest.mark.parametrize("feat,V", CASES)
def test_joint_lattice_blur_and_slice_parity(fr, ctx, feat, V, splat):
    p = synth.random_cloud_pair(51 + feat + V, 1777, 2501, feat=feat, residual=RES[V])
    _say(f"[blur] feat={feat} V={V} splat={splat} N={len(p.obs)} M={len(p.model)}")
    T = synth.random_motion(np.random.default_rng(feat + V + splat), np.radians(3.0), 0.01)
    mat = oracle.pose_to_mat12(T)
    xf = fr.XForm(fr.FR_XF_RIGID, torch.from_numpy(mat.copy()).cuda(), n_seg=1)
    obs = upload([p.obs], [p.obs_n])
    model = upload([p.model], [p.model_n])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(feat, V, p.sigma, p.sigma_n, splat), model=model, xf=xf)
    k = oracle.scale_factors(oracle.feature_sigmas(feat, p.sigma, p.sigma_n))
    x32 = oracle.transform_f32(mat, p.model)
    n32 = oracle.transform_f32(mat, p.model_n, translate=False)
    fx = oracle.features(x32, n32, feat)
    ref = oracle.joint_lattice(oracle.features(p.obs, p.obs_n, feat), oracle.splat_values(p.obs, p.obs_n, RES[V]),
                               fx, k)
    keys, occ, vals = lat.export(0)
    np.testing.assert_array_equal(keys, ref.keys)
    np.testing.assert_array_equal(occ, ref.occ)
    assert occ.sum() == (feat + 1) * (len(p.obs) + len(p.model))
    L = float(np.abs(p.obs).max())
    _close_vals(vals, ref.vals, L, "splat")
    lat.blur()
    rb = oracle.lattice_blur(ref)
    keys2, occ2, vals2 = lat.export(0)
    np.testing.assert_array_equal(keys2, ref.keys)
    np.testing.assert_array_equal(occ2, ref.occ)
    _close_vals(vals2, rb.vals, L, "blur")
    M = len(p.model)
    m0 = torch.empty(M, device="cuda")
    m1 = torch.empty(3 * M, device="cuda")
    ns = torch.empty(3 * M, device="cuda") if V == 7 else None
    fr.fr_estep(lat.h, model, xf, m0, m1, ns)
    torch.cuda.synchronize()
    g = oracle.lattice_slice(rb, fx)
    assert_estep_close(soa(m0), soa(m1).reshape(3, M).T, soa(ns).reshape(3, M).T if ns is not None else None,
                       g[:, 0], g[:, 1:4], g[:, 4:7] if V == 7 else None, float(rb.vals[:, 0].max()), L)
    assert (g[:, 0] > 0).all()   # every model point finds its own simplex
    lat.close()


def _register_blurred(fr, ctx, pairs, feat, res, iters, T0s, w):
    model = upload([q.model for q in pairs], [q.model_n for q in pairs])
    obs = upload([q.obs for q in pairs], [q.obs_n for q in pairs])
    q = pairs[0]
    prm = fr.register_params(feat, res, q.sigma, q.sigma_n, iters=iters, w=w, blurred=True)
    return fr.register(ctx, model, obs, prm, T0=np.stack(T0s))


def test_register_blurred_matches_the_oracle(fr, ctx):
    p = synth.ellipsoid_pair(4, m=2000, max_angle_deg=6, max_trans=0.03)
    _say(f"[blur-em] ellipsoid M={len(p.model)} N={len(p.obs)} 30 iterations")
    hist = []
    Tr = oracle.register_rigid_blurred(p.model, p.model_n, p.obs, p.obs_n, feat=3, residual="pt2pt", sigma=p.sigma,
                                       w=p.w, iters=30, T0=np.eye(4), history=hist)
    for k in (0, 5, 15):
        Tk = np.eye(4) if k == 0 else hist[k - 1]["T"]
        T1, st1, _ = _register_blurred(fr, ctx, [p], 3, "pt2pt", 1, [Tk], p.w)
        ang, dt, ok = pose_close(T1[0], hist[k]["T"])
        assert st1[0] == 0 and ok, (k, ang, dt)
    T, st, rep = _register_blurred(fr, ctx, [p], 3, "pt2pt", 30, [np.eye(4)], p.w)
    ang, dt, ok = pose_close(T[0], Tr, tol=1e-3)
    assert st[0] == 0 and ok, (ang, dt)
    assert oracle.alignment_error(T[0], p.T_gt, p.model) < 2e-3
    assert rep.iterations == 30


def test_register_blurred_batch_matches_oracle_and_alone(fr, ctx):
    pairs = [synth.depth_pair(70 + i, width=w, height=h, f=f)
             for i, (w, h, f) in enumerate([(160, 120, 131.25), (96, 72, 78.75)])]
    d = np.array([0.01, -0.01, 0.005, 0.01, 0.005, -0.01])
    T0s = [q.T_gt @ oracle.se3_exp(d * (1 + 0.3 * i)) for i, q in enumerate(pairs)]
    _say(f"[blur-batch] sizes={[len(q.model) for q in pairs]}")
    T1, st1, _ = _register_blurred(fr, ctx, pairs, 6, "pt2pl", 1, T0s, pairs[0].w)
    for i, q in enumerate(pairs):
        h = []
        oracle.register_rigid_blurred(q.model, q.model_n, q.obs, q.obs_n, feat=6, residual="pt2pl", sigma=q.sigma,
                                      sigma_n=q.sigma_n, w=q.w, iters=1, T0=T0s[i], history=h)
        ang, dt, ok = pose_close(T1[i], h[0]["T"])
        assert st1[i] == 0 and ok, (i, ang, dt)
    T, st, _ = _register_blurred(fr, ctx, pairs, 6, "pt2pl", 8, T0s, pairs[0].w)
    Ta, sta, _ = _register_blurred(fr, ctx, pairs[1:], 6, "pt2pl", 8, T0s[1:], pairs[0].w)
    np.testing.assert_array_equal(Ta[0], T[1])
    for i, q in enumerate(pairs):
        assert oracle.alignment_error(T[i], q.T_gt, q.model) < 2e-3


@pytest.mark.parametrize("case", ["ellipsoid", "depth", "depth_large"])
def test_register_blurred_rebuilt_in_place_equals_the_host_sized_build(fr, ctx, case):
    """fr_register with FR_BLURRED rebuilds the joint lattice in place every iteration (storage sized once;
    joint clouds of up to 2^17 incidences sum by vertex lists, larger ones sort; beyond 2^20 the host-sized
    build runs).  One iteration of it must equal, bitwise, the same iteration by hand: the host-sized joint
    build, its blur, the slice, the reduction and the solve."""
    if case == "ellipsoid":
        p = synth.ellipsoid_pair(6, m=2000, max_angle_deg=6, max_trans=0.03)
        feat, res, V = 3, "pt2pt", 4
    elif case == "depth":
        p = synth.depth_pair(71, width=160, height=120, f=131.25)
        feat, res, V = 6, "pt2pl", 7
    else:
        p = synth.depth_pair(72, width=320, height=240, f=262.5)
        feat, res, V = 6, "pt2pl", 7
    T0 = p.T_gt @ oracle.se3_exp(np.array([0.01, -0.01, 0.005, 0.01, 0.005, -0.01]))
    model = upload([p.model], [p.model_n] if feat == 6 else None)
    obs = upload([p.obs], [p.obs_n] if feat == 6 else None)
    _say(f"[blur-inplace] {case} M={len(p.model)} N={len(p.obs)} joint incidences={(feat + 1) * (model.n + obs.n)}")
    c, sigma = 0.37, float(p.sigma[0])
    prm = fr.register_params(feat, res, p.sigma, p.sigma_n, iters=1, c=c, blurred=True)
    T1, st1, _ = fr.register(ctx, model, obs, prm, T0=T0[None])
    assert st1[0] == 0
    # by hand, with the host-sized build
    mat = oracle.pose_to_mat12(T0)
    xf = fr.XForm(fr.FR_XF_RIGID, torch.from_numpy(mat.copy()).cuda(), n_seg=1)
    lat = fr.Lattice(ctx, obs, fr.lattice_params(feat, V, p.sigma, p.sigma_n), model=model, xf=xf)
    lat.blur()
    M = model.n
    m0, m1 = torch.empty(M, device="cuda"), torch.empty(3 * M, device="cuda")
    ns = torch.empty(3 * M, device="cuda") if V == 7 else None
    fr.fr_estep(lat.h, model, xf, m0, m1, ns)
    jtj = torch.zeros(21, dtype=torch.float64, device="cuda")
    jtr = torch.zeros(6, dtype=torch.float64, device="cuda")
    stt = torch.zeros(4, dtype=torch.float64, device="cuda")
    fr.fr_mstep_reduce(model, xf, m0, m1, ns, fr.FR_PT2PL if res == "pt2pl" else fr.FR_PT2PT, c, sigma, jtj, jtr,
                       stt)
    poses = torch.tensor(T0.reshape(-1), dtype=torch.float64, device="cuda")
    mats = torch.zeros(12, dtype=torch.float32, device="cuda")
    tn = torch.zeros(2, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    fr.fr_solve_rigid(1, jtj, jtr, poses, mats, tn, status)
    np.testing.assert_array_equal(T1[0], soa(poses).reshape(4, 4))
    lat.close()


def test_blurred_argument_errors(fr, ctx):
    p = synth.random_cloud_pair(5, 300, 300, feat=3, residual="pt2pt")
    obs, model = upload([p.obs]), upload([p.model])
    with pytest.raises(fr.FRError) as e:
        fr.register(ctx, model, obs, fr.register_params(3, "pt2pt", p.sigma, iters=2, blurred=True, fused=True))
    assert e.value.status == fr.FR_EINVAL
    mats = torch.zeros(12, device="cuda")
    seg = fr.XForm(fr.FR_XF_SEGMENTED, mats, seg_offsets=[0, len(p.model)])
    with pytest.raises(fr.FRError) as e:
        fr.Lattice(ctx, obs, fr.lattice_params(3, 4, p.sigma), model=model, xf=seg)
    assert e.value.status == fr.FR_EINVAL
    with pytest.raises(fr.FRError) as e:
        fr.Lattice(ctx, obs, fr.lattice_params(3, fr.FR_VAL_PT2PT_M2, p.sigma), model=model)
    assert e.value.status == fr.FR_EINVAL
    lat = fr.Lattice(ctx, obs, fr.lattice_params(3, fr.FR_VAL_PT2PT_M2, p.sigma))
    with pytest.raises(fr.FRError) as e:
        lat.blur()
    assert e.value.status == fr.FR_EINVAL
    lat.close()
