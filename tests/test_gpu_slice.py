"""The two slice kernels of the E-step (Sec. 4.2 slice; Eq. 6 / Eq. 9) and the context's autotuner.

FR_SLICE_SHARED looks each distinct vertex of a wavefront's 64 consecutive model points up once and sums
every point's vertices in the same order with the same arithmetic as FR_SLICE_PLAIN, so the two must agree
bitwise on every input: range-image frames (where neighbouring points share most vertices), clouds in no
order (where a wave has more distinct vertices than its LDS holds and takes the plain lookups), ragged
batches of several sets, every value layout.  Against the oracle the shared form is also checked directly.
"""
import numpy as np
import pytest

import oracle
import synth
from _helpers import assert_estep_close, oracle_lattice, soa, upload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

RES = {4: "pt2pt", 7: "pt2pl"}


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


def _estep(fr, ctx, lat, model, xf, V, slice_):
    fr.fr_ctx_set_tuning(ctx.h, slice_)
    M = model.n
    m0 = torch.full((M,), float("nan"), device="cuda")
    m1 = torch.full((3 * M,), float("nan"), device="cuda")
    ns = torch.full((3 * M,), float("nan"), device="cuda") if V == 7 else None
    fr.fr_estep(lat.h, model, xf, m0, m1, ns)
    torch.cuda.synchronize()
    return soa(m0), soa(m1), (soa(ns) if ns is not None else None)


def _both(fr, ctx, lat, model, xf, V):
    a = _estep(fr, ctx, lat, model, xf, V, fr.FR_SLICE_PLAIN)
    b = _estep(fr, ctx, lat, model, xf, V, fr.FR_SLICE_SHARED)
    for u, v in zip(a, b):
        if u is not None:
            assert not np.isnan(v).any()
            np.testing.assert_array_equal(u.view(np.uint32), v.view(np.uint32))
    return b


def _rigid(fr, Ts):
    mats = np.concatenate([oracle.pose_to_mat12(T) for T in Ts]).astype(np.float32)
    return fr.XForm(fr.FR_XF_RIGID, torch.from_numpy(mats).cuda())


@pytest.mark.parametrize("feat,V", [(3, 4), (3, 7), (6, 4), (6, 7)])
def test_shared_slice_is_bitwise_plain_on_depth_frames(fr, ctx, feat, V):
    # two small depth frames of different sizes (ragged waves and tiles), moved by their start poses
    pairs = [synth.depth_pair(s, width=160, height=120, f=131.25) for s in (4, 5)]
    _say(f"[slice-depth] feat={feat} V={V} M={[len(p.model) for p in pairs]}")
    p0 = pairs[0]
    obs = upload([p.obs for p in pairs], [p.obs_n for p in pairs])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(feat, V, p0.sigma, p0.sigma_n))
    model = upload([p.model for p in pairs], [p.model_n for p in pairs])
    Ts = [p.T_gt @ oracle.se3_exp(np.array([0.01, -0.01, 0.005, 0.003, 0.0, -0.002])) for p in pairs]
    m0, m1, ns = _both(fr, ctx, lat, model, _rigid(fr, Ts), V)
    # the shared form against the oracle, set by set
    off = model.offsets
    for s, (p, T) in enumerate(zip(pairs, Ts)):
        ref = oracle_lattice(p.obs, p.obs_n, feat, RES[V], p.sigma, p.sigma_n)
        mat = oracle.pose_to_mat12(T).astype(np.float32)
        x32 = oracle.transform_f32(mat, p.model)
        n32 = oracle.transform_f32(mat, p.model_n, translate=False) if feat == 6 else None
        g = oracle.lattice_slice(ref, oracle.features(x32, n32, feat))
        lo, hi = int(off[s]), int(off[s + 1])
        M = model.n
        mm1 = m1.reshape(3, M)[:, lo:hi].T
        mns = ns.reshape(3, M)[:, lo:hi].T if ns is not None else None
        assert_estep_close(m0[lo:hi], mm1, mns, g[:, 0], g[:, 1:4], g[:, 4:7] if V == 7 else None,
                           float(ref.vals[:, 0].max()), float(np.abs(p.obs).max()))
    lat.close()


def test_shared_slice_on_points_in_no_order(fr, ctx):
    # an ellipsoid sampled at random: neighbouring indices are far apart, most waves hold more distinct
    # vertices than their LDS and take the plain lookups; results are still bitwise those of the plain form
    p = synth.ellipsoid_pair(3, m=5000)
    _say(f"[slice-random] M={len(p.model)}")
    obs = upload([p.obs])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(3, 4, p.sigma))
    model = upload([p.model])
    _both(fr, ctx, lat, model, _rigid(fr, [p.T_gt]), 4)
    # the same cloud sorted along one axis: some waves share, some do not
    order = np.argsort(p.model[:, 0] * 1000.0 + p.model[:, 1])
    _both(fr, ctx, lat, upload([p.model[order]]), _rigid(fr, [p.T_gt]), 4)
    lat.close()


def test_shared_slice_tails_and_empty_sets(fr, ctx):
    # sets of 1, 63, 64, 65, 0 and 300 points cut from one depth frame: waves with one live lane, a full
    # wave, one lane over, an empty set, and a ragged last tile
    p = synth.depth_pair(6, width=160, height=120, f=131.25)
    sizes = [1, 63, 64, 65, 0, 300]
    starts = np.cumsum([0] + sizes[:-1]) + 500
    sets = [p.model[a:a + n] for a, n in zip(starts, sizes)]
    nsets = [p.model_n[a:a + n] for a, n in zip(starts, sizes)]
    _say(f"[slice-tails] sizes={sizes}")
    obs = upload([p.obs] * len(sizes), [p.obs_n] * len(sizes))
    lat = fr.Lattice(ctx, obs, fr.lattice_params(6, 7, p.sigma, p.sigma_n))
    model = upload(sets, nsets)
    _both(fr, ctx, lat, model, _rigid(fr, [p.T_gt] * len(sizes)), 7)
    _both(fr, ctx, lat, model, fr.XForm(), 7)
    lat.close()


def test_shared_slice_second_moment_layouts(fr, ctx):
    # the |y|^2 layouts of the variance update: the second moment about the target reads every vertex's
    # values again after the sums
    p = synth.depth_pair(7, width=160, height=120, f=131.25)
    for feat, V in [(3, 5), (6, 8)]:
        _say(f"[slice-m2] feat={feat} V={V}")
        lat = fr.Lattice(ctx, upload([p.obs], [p.obs_n]), fr.lattice_params(feat, V, p.sigma, p.sigma_n))
        model = upload([p.model], [p.model_n])
        M = model.n
        outs = []
        for sl in (fr.FR_SLICE_PLAIN, fr.FR_SLICE_SHARED):
            fr.fr_ctx_set_tuning(ctx.h, sl)
            m0, m1 = torch.empty(M, device="cuda"), torch.empty(3 * M, device="cuda")
            ns = torch.empty(3 * M, device="cuda") if V == 8 else None
            m2 = torch.empty(M, device="cuda")
            fr.fr_estep_m2(lat.h, model, _rigid(fr, [p.T_gt]), m0, m1, ns, m2)
            torch.cuda.synchronize()
            outs.append([soa(t) for t in (m0, m1, m2) + ((ns,) if ns is not None else ())])
        for u, v in zip(*outs):
            np.testing.assert_array_equal(u.view(np.uint32), v.view(np.uint32))
        lat.close()


def test_autotuner_records_its_choice(fr, ctx):
    # FR_SLICE_AUTO: the first E-step of a (d, V, transform, size class) times both forms and keeps the
    # faster; the outputs are those of either form
    p = synth.depth_pair(8, width=320, height=240, f=262.5)
    _say(f"[autotune] M={len(p.model)}")
    lat = fr.Lattice(ctx, upload([p.obs], [p.obs_n]), fr.lattice_params(6, 7, p.sigma, p.sigma_n))
    model = upload([p.model], [p.model_n])
    xf = _rigid(fr, [p.T_gt])
    ref = _estep(fr, ctx, lat, model, xf, 7, fr.FR_SLICE_PLAIN)
    assert fr.fr_ctx_tuning_table(ctx.h) == []
    auto = _estep(fr, ctx, lat, model, xf, 7, fr.FR_SLICE_AUTO)
    for u, v in zip(ref, auto):
        np.testing.assert_array_equal(u.view(np.uint32), v.view(np.uint32))
    tab = fr.fr_ctx_tuning_table(ctx.h)
    assert len(tab) == 1
    e = tab[0]
    assert (e["d"], e["V"], e["xf_kind"]) == (6, 7, fr.FR_XF_RIGID)
    assert 2 ** e["size_class"] <= 256 * ((len(p.model) + 255) // 256) < 2 ** (e["size_class"] + 1)
    assert e["us_plain"] > 0 and e["us_shared"] > 0
    assert e["slice"] == (fr.FR_SLICE_SHARED if e["us_shared"] < e["us_plain"] else fr.FR_SLICE_PLAIN)
    _say(f"[autotune] {e}")
    # a second launch of the same class reuses the entry
    _estep(fr, ctx, lat, model, xf, 7, fr.FR_SLICE_AUTO)
    assert len(fr.fr_ctx_tuning_table(ctx.h)) == 1
    lat.close()
