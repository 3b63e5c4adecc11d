"""Lattices rebuilt in place (Sec. 3.3: the optimised variance rebuilds the lattice of Sec. 3.2 every iteration).

fr_lattice_build_inplace sizes its storage once from the observation cloud and fr_lattice_rebuild refills it at
new per-set scales without a host wait.  Its tables hold what fr_lattice_build makes at the same scale, so the
E-step (Eq. 6, Eq. 9 and the |y|^2 channel of the variance update) on either lattice must agree bitwise with
the sorted splat, and within binary32 atomic rounding with the atomic one; set s rebuilt at its own scale must
match a lattice of that set alone built at that scale.  Against the oracle the in-place lattice is checked
directly as well.
"""
import numpy as np
import pytest

import oracle
import synth
from _helpers import assert_estep_close, assert_lattice_equal, oracle_lattice, soa, upload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

RES = {4: "pt2pt", 5: "pt2pt", 7: "pt2pl", 8: "pt2pl"}


@pytest.fixture(scope="module")
def fr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1811_10136_amd as fr
    return fr


@pytest.fixture()
def ctx(fr):
    c = fr.Context(0)
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)


def _estep(fr, lat_h, model, mats, V):
    M = model.n
    m0 = torch.full((M,), float("nan"), device="cuda")
    m1 = torch.full((3 * M,), float("nan"), device="cuda")
    ns = torch.full((3 * M,), float("nan"), device="cuda") if V in (7, 8) else None
    xf = fr.XForm(fr.FR_XF_RIGID, torch.from_numpy(mats).cuda())
    if V in (5, 8):
        m2 = torch.full((M,), float("nan"), device="cuda")
        fr.fr_estep_m2(lat_h, model, xf, m0, m1, ns, m2)
    else:
        m2 = None
        fr.fr_estep(lat_h, model, xf, m0, m1, ns)
    torch.cuda.synchronize()
    return [soa(t) for t in (m0, m1, ns, m2) if t is not None]


def _mats(Ts):
    return np.concatenate([oracle.pose_to_mat12(T) for T in Ts]).astype(np.float32)


def _pairs(small=False):
    # two range-image frames: ragged tiles, shared simplices.  Small frames keep a rebuild under 2^17
    # incidences, where the per-vertex sums walk vertex lists instead of sorting the partial records.
    if small:
        return [synth.depth_pair(s, width=64, height=48, f=52.5) for s in (11, 12)]
    return [synth.depth_pair(s, width=160, height=120, f=131.25) for s in (11, 12)]


@pytest.mark.parametrize("small", [False, True])
@pytest.mark.parametrize("feat,V,splat", [(3, 4, 0), (3, 5, 0), (6, 7, 0), (6, 8, 0), (6, 8, 1), (3, 5, 1)])
def test_rebuild_matches_a_fresh_build(fr, ctx, feat, V, splat, small):
    pairs = _pairs(small)
    p0 = pairs[0]
    obs = upload([p.obs for p in pairs], [p.obs_n for p in pairs])
    model = upload([p.model for p in pairs], [p.model_n for p in pairs])
    mats = _mats([p.T_gt for p in pairs])
    _say(f"[inplace] feat={feat} V={V} splat={splat} M={model.n} incidences={obs.n * (feat + 1)}")
    prm = fr.lattice_params(feat, V, p0.sigma, p0.sigma_n, splat)
    lat = fr.fr_lattice_build_inplace(ctx.h, obs, prm, None)
    try:
        # the build at the parameters' scale, then rebuilds at other scales and back
        for sig in (None, 0.7 * p0.sigma[0], 1.6 * p0.sigma[0], None):
            if sig is not None:
                fr.fr_lattice_rebuild(lat, [sig, sig])
                s3 = (sig, sig, sig)
            else:
                fr.fr_lattice_rebuild(lat, [p0.sigma[0]] * 2)
                s3 = tuple(p0.sigma)
            fr.fr_sync_status(lat)
            ref = fr.Lattice(ctx, obs, fr.lattice_params(feat, V, s3, p0.sigma_n, splat))
            a = _estep(fr, lat, model, mats, V)
            b = _estep(fr, ref.h, model, mats, V)
            ref.close()
            for u, v in zip(a, b):
                assert not np.isnan(u).any()
                if splat == 0:
                    np.testing.assert_array_equal(u.view(np.uint32), v.view(np.uint32))
                else:
                    np.testing.assert_allclose(u, v, rtol=1e-5, atol=1e-6 * max(1.0, float(np.abs(v).max())))
    finally:
        fr.fr_lattice_destroy(lat)


def test_per_set_scales_match_each_set_alone(fr, ctx):
    # two sets rebuilt at different scales: each set's slice equals that of its own lattice at its scale
    pairs = _pairs()
    obs = upload([p.obs for p in pairs], [p.obs_n for p in pairs])
    model = upload([p.model for p in pairs], [p.model_n for p in pairs])
    mats = _mats([p.T_gt for p in pairs])
    sig = [0.021, 0.034]
    _say(f"[inplace-sets] sigma={sig}")
    prm = fr.lattice_params(6, 8, pairs[0].sigma, pairs[0].sigma_n)
    lat = fr.fr_lattice_build_inplace(ctx.h, obs, prm, sig)
    try:
        got = _estep(fr, lat, model, mats, 8)
        off = model.offsets
        for s, p in enumerate(pairs):
            o1, m1 = upload([p.obs], [p.obs_n]), upload([p.model], [p.model_n])
            ref = fr.Lattice(ctx, o1, fr.lattice_params(6, 8, (sig[s],) * 3, p.sigma_n))
            want = _estep(fr, ref.h, m1, _mats([p.T_gt]), 8)
            ref.close()
            lo, hi = int(off[s]), int(off[s + 1])
            M = model.n
            cuts = [lambda a: a[lo:hi], lambda a: a.reshape(3, M)[:, lo:hi].ravel(),
                    lambda a: a.reshape(3, M)[:, lo:hi].ravel(), lambda a: a[lo:hi]]
            for cut, u, v in zip(cuts, got, want):
                np.testing.assert_array_equal(cut(u).view(np.uint32), v.view(np.uint32))
    finally:
        fr.fr_lattice_destroy(lat)


def test_inplace_lattice_against_the_oracle(fr, ctx):
    p = synth.depth_pair(13, width=160, height=120, f=131.25)
    obs, model = upload([p.obs], [p.obs_n]), upload([p.model], [p.model_n])
    sig = 0.8 * p.sigma[0]
    _say(f"[inplace-oracle] M={len(p.model)} sigma={sig:.4f}")
    lat = fr.fr_lattice_build_inplace(ctx.h, obs, fr.lattice_params(6, 7, p.sigma, p.sigma_n), None)
    try:
        fr.fr_lattice_rebuild(lat, [sig])
        mat = _mats([p.T_gt])
        m0, m1, ns = _estep(fr, lat, model, mat, 7)
        ref = oracle_lattice(p.obs, p.obs_n, 6, "pt2pl", (sig,) * 3, p.sigma_n)
        x32 = oracle.transform_f32(mat, p.model)
        n32 = oracle.transform_f32(mat, p.model_n, translate=False)
        g = oracle.lattice_slice(ref, oracle.features(x32, n32, 6))
        M = model.n
        assert_estep_close(m0, m1.reshape(3, M).T, ns.reshape(3, M).T, g[:, 0], g[:, 1:4], g[:, 4:7],
                           float(ref.vals[:, 0].max()), float(np.abs(p.obs).max()))
    finally:
        fr.fr_lattice_destroy(lat)


def test_inplace_lattice_refuses_what_it_does_not_hold(fr, ctx):
    p = synth.depth_pair(14, width=64, height=48, f=52.5)
    obs = upload([p.obs], [p.obs_n])
    prm = fr.lattice_params(6, 7, p.sigma, p.sigma_n)
    lat = fr.fr_lattice_build_inplace(ctx.h, obs, prm, None)
    plain = fr.Lattice(ctx, obs, prm)
    try:
        with pytest.raises(fr.FRError):
            fr.fr_lattice_stats(lat, 0)
        with pytest.raises(fr.FRError):
            fr.fr_lattice_blur(lat)
        with pytest.raises(fr.FRError):
            fr.fr_lattice_rebuild(plain.h, [0.03])
        with pytest.raises(fr.FRError):
            fr.fr_lattice_rebuild(lat, [-1.0])
    finally:
        plain.close()
        fr.fr_lattice_destroy(lat)


def test_one_shot_build_of_a_set_beyond_two_sort_passes(fr, ctx):
    """A full 640x480 frame at sigma 0.02 m has about 322k vertices in one set, more than the 2^18 that the
    one-shot build's two 9-bit passes over per-set vertex ids cover, so its sort takes a third pass.  The
    lattice equals the oracle's (keys and counts exactly), and its slice is bitwise that of the in-place build,
    which sorts the same records by global vertex id in 8-bit passes."""
    p = synth.depth_pair(0)
    sig = 0.02
    obs = upload([p.obs], [p.obs_n])
    model = upload([p.model], [p.model_n])
    prm = fr.lattice_params(6, 7, (sig, sig, sig), p.sigma_n, 0)
    lat = fr.Lattice(ctx, obs, prm)
    res = None
    try:
        nv = lat.stats(0)[0]
        _say(f"[sort-3-pass] {len(p.obs)} observation points, {nv} vertices")
        assert nv > 1 << 18
        keys, occ, vals = lat.export(0)
        ref = oracle_lattice(p.obs, p.obs_n, 6, "pt2pl", (sig, sig, sig), p.sigma_n)
        assert_lattice_equal(keys, occ, vals, ref, float(np.abs(p.obs).max()))
        res = fr.fr_lattice_build_inplace(ctx.h, obs, prm, None)
        fr.fr_lattice_rebuild(res, [sig])
        fr.fr_sync_status(res)
        mats = _mats([p.T_gt])
        a = _estep(fr, res, model, mats, 7)
        b = _estep(fr, lat.h, model, mats, 7)
        for u, v in zip(a, b):
            np.testing.assert_array_equal(u.view(np.uint32), v.view(np.uint32))
    finally:
        if res is not None:
            fr.fr_lattice_destroy(res)
        lat.close()
