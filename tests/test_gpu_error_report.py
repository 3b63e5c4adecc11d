"""Error of each result of the binary32 / binary64 path against the binary64 oracle, stated per result.

Values, slice outputs and per-tile sums are binary32 on the GPU; the vertex sums of the sorted splat, the
tile-to-segment sums, the solve and the pose update are binary64.  For one 640x480 depth frame (d = 6,
point-to-plane: the pairs of the benchmark batch), one ellipsoid (d = 3, point-to-point) and the optimised
variance, this module measures the error of every result against the oracle on the same inputs and
prints it ("[error] ..." lines, collected with pytest -s): lattice values, M0 / M1 / N of the slice, the
normal equations A and b, and the pose (and scale) after the registration's iterations.  Each is also held
to the bound the parity tests use, so the table below is what those bounds leave room for.
"""
import numpy as np
import pytest

import oracle
import synth
from _helpers import abs_scales, oracle_lattice, pose_close, soa, upload, upper

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


def _report(name, value, bound):
    print(f"[error] {name}: {value:.3e} (bound {bound:.0e})", flush=True)
    assert value <= bound, (name, value, bound)


def test_depth_frame_lattice_slice_and_normal_equations(fr, ctx):
    p = synth.depth_pair(3)
    print(f"[error] depth frame: model {len(p.model)}, observation {len(p.obs)} points", flush=True)
    obs, model = upload([p.obs], [p.obs_n]), upload([p.model], [p.model_n])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(6, 7, p.sigma, p.sigma_n, 0))
    ref = oracle_lattice(p.obs, p.obs_n, 6, "pt2pl", p.sigma, p.sigma_n)
    keys, occ, vals = lat.export(0)
    np.testing.assert_array_equal(keys, ref.keys)
    np.testing.assert_array_equal(occ, ref.occ)
    rv = ref.vals
    scale = np.maximum(1.0, np.abs(rv[:, :1]))   # channel error relative to the vertex weight (>= 1 incidence)
    L = float(np.abs(p.obs).max())
    e_w = float((np.abs(vals[:, 0] - rv[:, 0]) / scale[:, 0]).max())
    e_y = float((np.abs(vals[:, 1:4] - rv[:, 1:4]) / (scale * L)).max())
    e_n = float((np.abs(vals[:, 4:7] - rv[:, 4:7]) / scale).max())
    _report("lattice weight sum W_v, |dW| / max(1, W)", e_w, 1e-5 * 64)
    _report("lattice sum of b y, |d| / (max(1, W) max|y|)", e_y, 1e-5 * 64)
    _report("lattice sum of b n, |d| / max(1, W)", e_n, 1e-5 * 64)

    T = p.T_gt @ oracle.se3_exp(np.array([0.003, -0.002, 0.001, 0.004, 0.002, -0.003]))
    mat = oracle.pose_to_mat12(T)
    M = len(p.model)
    xf = fr.XForm(fr.FR_XF_RIGID, torch.from_numpy(mat.copy()).cuda(), n_seg=1)
    m0, m1, ns = (torch.empty(M, device="cuda"), torch.empty(3 * M, device="cuda"),
                  torch.empty(3 * M, device="cuda"))
    fr.fr_estep(lat.h, model, xf, m0, m1, ns)
    g0, g1, gn = soa(m0).astype(np.float64), soa(m1).reshape(3, M).T.astype(np.float64), \
        soa(ns).reshape(3, M).T.astype(np.float64)
    x32 = oracle.transform_f32(mat, p.model)
    n32 = oracle.transform_f32(mat, p.model_n, translate=False)
    g = oracle.lattice_slice(ref, oracle.features(x32, n32, 6))
    vmax = float(rv[:, 0].max())
    floor = 1e-6 * vmax
    sup = g[:, 0] > floor
    e0 = float((np.abs(g0 - g[:, 0]) / (g[:, 0] + floor)).max())
    e0_abs = float(np.abs(g0 - g[:, 0]).max() / vmax)
    e1 = float((np.abs(g1 - g[:, 1:4]).max(axis=1) / ((g[:, 0] + floor) * L)).max())
    en = float((np.abs(gn - g[:, 4:7]).max(axis=1) / (g[:, 0] + floor)).max())
    print(f"[error] slice: {int(sup.sum())} of {M} model points supported", flush=True)
    _report("slice M0, |dM0| / (M0 + 1e-6 max W_v)", e0, 1e-5 + 1e-6)
    _report("slice M0, |dM0| / max W_v", e0_abs, 1e-5)
    _report("slice M1, |dM1| / ((M0 + 1e-6 max W_v) max|y|)", e1, 1e-5 + 1e-6)
    _report("slice N, |dN| / (M0 + 1e-6 max W_v)", en, 1e-5 + 1e-6)

    # normal equations from the GPU's own slice outputs, on both sides
    c, sigma = 0.37, float(p.sigma[0])
    jtj = torch.zeros(21, dtype=torch.float64, device="cuda")
    jtr = torch.zeros(6, dtype=torch.float64, device="cuda")
    st = torch.zeros(4, dtype=torch.float64, device="cuda")
    fr.fr_mstep_reduce(model, xf, m0, m1, ns, fr.FR_PT2PL, c, sigma, jtj, jtr, st)
    R = mat.reshape(3, 4).astype(np.float64)
    x64 = p.model.astype(np.float64) @ R[:, :3].T + R[:, 3]
    m0f, m1f, nsf = soa(m0), soa(m1).reshape(3, M).T, soa(ns).reshape(3, M).T
    A, b, _ = oracle.normal_equations(x64, m0f, m1f, nsf, c, sigma, "pt2pl")
    sA, sb = abs_scales(x64, m0f, m1f, nsf, c, sigma, "pt2pl")
    eA = float((np.abs(soa(jtj) - upper(A)) / upper(sA)).max())
    eb = float((np.abs(soa(jtr) - b) / sb).max())
    _report("normal equations A, |dA| / sum|w J^T J| per entry", eA, 1e-5)
    _report("normal equations b, |db| / sum|w J^T r| per entry", eb, 1e-5)
    lat.close()


def test_registration_poses(fr, ctx):
    p = synth.depth_pair(3)
    T0 = p.T_gt @ oracle.se3_exp(np.array([0.01, -0.01, 0.005, 0.01, 0.005, -0.01]))
    prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=20, w=p.w)
    T, st, _ = fr.register(ctx, upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n]), prm, T0=T0[None])
    ref = oracle.register_rigid(p.model, p.model_n, p.obs, p.obs_n, feat=6, residual="pt2pl", sigma=p.sigma,
                                sigma_n=p.sigma_n, w=p.w, iters=20, T0=T0)
    ang, dt, _ = pose_close(T[0], ref)
    assert st[0] == 0
    _report("depth frame, 20 iterations: pose rotation (rad)", ang, 1e-4)
    _report("depth frame, 20 iterations: pose translation (m)", dt, 1e-4)
    # the same registration with the slice and the reduction in one kernel (the benchmark's step)
    prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=20, w=p.w, fused=True)
    T, st, _ = fr.register(ctx, upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n]), prm, T0=T0[None])
    ang, dt, _ = pose_close(T[0], ref)
    assert st[0] == 0
    _report("depth frame, 20 iterations, fused slice + reduction: pose rotation (rad)", ang, 1e-4)
    _report("depth frame, 20 iterations, fused slice + reduction: pose translation (m)", dt, 1e-4)

    e = synth.ellipsoid_pair(1)
    T0 = e.T_gt @ oracle.se3_exp(np.array([0.01, -0.01, 0.005, 0.004, 0.0, -0.003]))
    prm = fr.register_params(3, "pt2pt", e.sigma, iters=e.iters, w=e.w)
    T, st, _ = fr.register(ctx, upload([e.model]), upload([e.obs]), prm, T0=T0[None])
    ref = oracle.register_rigid(e.model, None, e.obs, None, feat=3, residual="pt2pt", sigma=e.sigma, w=e.w,
                                iters=e.iters, T0=T0)
    ang, dt, _ = pose_close(T[0], ref)
    _report(f"ellipsoid, {e.iters} iterations: pose rotation (rad)", ang, 1e-4)
    _report(f"ellipsoid, {e.iters} iterations: pose translation (units)", dt, 1e-4)


def test_optimised_variance_pose_and_scale(fr, ctx):
    p = synth.depth_pair(0)
    T0 = p.T_gt @ oracle.se3_exp(np.array([0.01, -0.01, 0.005, 0.01, 0.005, -0.01]))
    iters = 8
    Tr, sr = oracle.register_rigid_sigma(p.model, p.model_n, p.obs, p.obs_n, feat=6, residual="pt2pl",
                                         sigma0=p.sigma[0], sigma_min=0.002, sigma_n=p.sigma_n, w=p.w, iters=iters,
                                         T0=T0)
    prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=iters, w=p.w, m2=True)
    T, s, st, _ = fr.register_sigma(ctx, upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n]), prm,
                                    p.sigma[0], 0.002, T0=T0[None])
    ang, dt, _ = pose_close(T[0], Tr)
    _report(f"optimised variance, depth frame, {iters} iterations: pose rotation (rad)", ang, 1e-4)
    _report(f"optimised variance, depth frame, {iters} iterations: pose translation (m)", dt, 1e-4)
    _report(f"optimised variance, depth frame, {iters} iterations: scale s, relative", abs(s[0] / sr - 1.0), 1e-3)
