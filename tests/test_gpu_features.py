"""GPU parity of the descriptor E-step (Sec. 3.3 "Features", Eq. 8) and the registration by descriptors,
against the oracle, for descriptors of 8, 16 and 32 dimensions.

Tolerances as _helpers.py: keys and occupancy bit-exact, vertex values and slices to the binary32 weight
rounding; poses (fixed targets, so a well-conditioned loop) to 1e-4.
"""
import numpy as np
import pytest

import oracle
import synth
from _helpers import assert_estep_close, pose_close, soa, upload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DIMS = [8, 16, 32]


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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("splat", [0, 1], ids=["sorted", "atomic"])
@pytest.mark.parametrize("dim", DIMS)
def test_feature_lattice_and_estep_parity(fr, ctx, dim, splat):
    p = synth.feature_pair(80 + dim, m=2500, dim=dim)
    e = p.extra
    _say(f"[feat] dim={dim} splat={splat} M={len(p.model)} N={len(p.obs)}")
    obs, model = upload([p.obs]), upload([p.model])
    of, mf = _dev(e["obs_feat"]), _dev(e["model_feat"])
    lat = fr.FeatureLattice(ctx, obs, of, e["sigma_f"], splat)
    ref = oracle.feature_lattice(p.obs, e["obs_feat"], e["sigma_f"])
    keys, occ, vals = lat.export(0)
    np.testing.assert_array_equal(keys, ref.keys)
    np.testing.assert_array_equal(occ, ref.occ)
    assert occ.sum() == (dim + 1) * len(p.obs)
    L = float(np.abs(p.obs).max())
    scale = np.maximum(1.0, np.abs(ref.vals[:, :1]))
    tol = 1e-5 * scale * np.array([1.0, L, L, L])[None, :]
    err = np.abs(vals.astype(np.float64) - ref.vals)
    assert (err <= tol).all(), f"{(err > tol).sum()} vertex values off; worst {err.max():.3e}"
    M = len(p.model)
    m0 = torch.empty(M, device="cuda")
    m1 = torch.empty(3 * M, device="cuda")
    fr.fr_estep_features(lat.h, model, mf, m0, m1)
    torch.cuda.synchronize()
    g = oracle.lattice_slice(ref, e["model_feat"])
    assert_estep_close(soa(m0), soa(m1).reshape(3, M).T, None, g[:, 0], g[:, 1:4], None, float(ref.vals[:, 0].max()),
                       L)
    assert (g[:, 0] > 0).mean() > 0.5
    lat.close()


def _register(fr, ctx, pairs, dim, iters, T0s=None, fixed=True):
    model = upload([q.model for q in pairs])
    obs = upload([q.obs for q in pairs])
    mf = _dev(np.concatenate([q.extra["model_feat"] for q in pairs]))
    of = _dev(np.concatenate([q.extra["obs_feat"] for q in pairs]))
    prm = fr.register_params(3, "pt2pt", 0.01, iters=iters, w=pairs[0].w, fixed=fixed)
    theta = np.repeat(np.eye(4)[None], len(pairs), 0) if T0s is None else np.stack(T0s).copy()
    st, rep = fr.fr_register_features(ctx.h, model, mf, obs, of, dim, pairs[0].extra["sigma_f"], prm, theta)
    return theta, st, rep


@pytest.mark.parametrize("dim", DIMS)
def test_register_features_matches_the_oracle_from_any_pose(fr, ctx, dim):
    p = synth.feature_pair({8: 97, 16: 92, 32: 90}[dim], m=6000, dim=dim)   # rotations of 130-150 degrees
    e = p.extra
    ang0 = np.degrees(oracle.rotation_angle(p.T_gt[:3, :3]))
    _say(f"[feat-em] dim={dim} rotation={ang0:.0f} deg")
    assert ang0 > 100
    T, st, rep = _register(fr, ctx, [p], dim, 20)
    Tr = oracle.register_rigid_features(p.model, e["model_feat"], p.obs, e["obs_feat"], sigma_f=e["sigma_f"], w=p.w,
                                        iters=20)
    ang, dt, ok = pose_close(T[0], Tr)
    assert st[0] == 0 and ok, (ang, dt)
    # 8-dimensional descriptors are less distinctive: more ambiguous matches pull the targets
    assert oracle.alignment_error(T[0], p.T_gt, p.model) < (5e-3 if dim == 8 else 1e-3)
    assert rep.iterations == 20


def test_register_features_batch_matches_oracle_and_alone(fr, ctx):
    pairs = [synth.feature_pair(100 + i, m=m, dim=16) for i, m in enumerate([4000, 1500, 7000])]
    _say(f"[feat-batch] sizes={[len(q.model) for q in pairs]}")
    T, st, _ = _register(fr, ctx, pairs, 16, 15)
    assert (st == 0).all()
    for i, q in enumerate(pairs):
        e = q.extra
        Tr = oracle.register_rigid_features(q.model, e["model_feat"], q.obs, e["obs_feat"], sigma_f=e["sigma_f"],
                                            w=q.w, iters=15)
        ang, dt, ok = pose_close(T[i], Tr)
        assert ok, (i, ang, dt)
    Ta, sta, _ = _register(fr, ctx, pairs[1:2], 16, 15)
    np.testing.assert_array_equal(Ta[0], T[1])
    # stopping on the twist ends every set at its own iteration
    Tt, stt, rep = _register(fr, ctx, pairs, 16, 40, fixed=False)
    assert rep.iterations < 40
    for i, q in enumerate(pairs):
        assert oracle.alignment_error(Tt[i], q.T_gt, q.model) < 1e-3


def test_feature_argument_errors(fr, ctx):
    p = synth.feature_pair(3, m=800, dim=16)
    obs, model = upload([p.obs]), upload([p.model])
    of = _dev(p.extra["obs_feat"])
    with pytest.raises(fr.FRError) as e:
        fr.fr_lattice_build_features(ctx.h, obs, _dev(np.zeros((len(p.obs), 12))), 12, 0.05)
    assert e.value.status == fr.FR_EINVAL
    with pytest.raises(fr.FRError) as e:
        fr.fr_lattice_build_features(ctx.h, obs, of, 16, 0.0)
    assert e.value.status == fr.FR_EINVAL
    flat = _dev(np.zeros(len(p.obs) * 16 + 1))
    with pytest.raises(fr.FRError) as e:                       # rows not 16-byte aligned
        fr.fr_lattice_build_features(ctx.h, obs, flat[1:], 16, 0.05)
    assert e.value.status == fr.FR_EINVAL
    lat = fr.FeatureLattice(ctx, obs, of, 0.05)
    M = len(p.model)
    m0, m1 = torch.empty(M, device="cuda"), torch.empty(3 * M, device="cuda")
    with pytest.raises(fr.FRError) as e:                       # the position slice does not take descriptor lattices
        fr.fr_estep(lat.h, model, fr.XForm(), m0, m1)
    assert e.value.status == fr.FR_EINVAL
    with pytest.raises(fr.FRError) as e:
        fr.fr_lattice_blur(lat.h)
    assert e.value.status == fr.FR_EINVAL
    lat.close()
    plain = fr.Lattice(ctx, obs, fr.lattice_params(3, 4, 0.02))
    with pytest.raises(fr.FRError) as e:                       # and the descriptor slice needs a descriptor lattice
        fr.fr_estep_features(plain.h, model, _dev(p.extra["model_feat"]), m0, m1)
    assert e.value.status == fr.FR_EINVAL
    plain.close()
