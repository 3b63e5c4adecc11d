"""End-to-end pins of the oracle's rigid EM loop (Sec. 3.1, Sec. 5).

Exact recovery: on noise-free, well-separated points each model point shares
lattice vertices only with its own observation (checked by brute force), so
M1/M0 is the exact correspondence and Gauss-Newton must land on the known motion.
"""
import numpy as np
import pytest

import oracle
import synth


def _kernel_matrix(p, T):
    feat = p.feat
    k = oracle.scale_factors(oracle.feature_sigmas(feat, p.sigma, p.sigma_n))
    mat = oracle.pose_to_mat12(T)
    x = oracle.transform_f32(mat, p.model)
    n = oracle.transform_f32(mat, p.model_n, translate=False)
    fy = oracle.features(p.obs, p.obs_n, feat)
    fx = oracle.features(x, n, feat)
    return oracle.brute_force_lattice_sum(fy, np.eye(len(p.obs)), fx, k)


@pytest.mark.parametrize("feat,residual", [(3, "pt2pt"), (6, "pt2pl"), (3, "pt2pl")])
def test_exact_recovery_on_separated_points(feat, residual):
    p = synth.separated_pair(4, 300, feat=feat, residual=residual)
    T0 = p.extra["T0"]
    for T in (T0, p.T_gt):
        K = _kernel_matrix(p, T)
        off = K - np.diag(np.diag(K))
        assert np.all(off == 0.0), "points are not separated beyond the kernel support"
        assert (np.diag(K) > 0).mean() > 0.95
    hist = []
    T = oracle.register_rigid(p.model, p.model_n, p.obs, p.obs_n, feat=feat, residual=residual, sigma=p.sigma,
                              sigma_n=p.sigma_n, c=0.0, iters=12, T0=T0, history=hist)
    assert np.abs(T - p.T_gt).max() < 1e-6
    assert oracle.alignment_error(T, p.T_gt, p.model) < 1e-6
    assert oracle.alignment_error(T0, p.T_gt, p.model) > 1e-3
    # Gauss-Newton with exact correspondences converges fast: last steps are tiny
    assert np.linalg.norm(hist[-1]["dz"]) < 1e-7


def test_ellipsoid_workload_runs_and_keeps_invariants():
    p = synth.ellipsoid_pair(0)
    assert p.model.shape == (2000, 3) and p.obs.shape == (2200, 3)
    lat = oracle.build_observation_lattice(p.obs, None, 3, "pt2pt", p.sigma, p.sigma_n)
    assert lat.occ.sum() == 4 * 2200
    np.testing.assert_allclose(lat.vals[:, 0].sum(), 2200.0, rtol=1e-12)
    # start close to the answer so that the E-step has support (30 deg is far outside
    # the 2-sigma basin of a sigma = 0.02 kernel on a unit-size cloud)
    T0 = p.T_gt @ oracle.se3_exp(np.array([0.01, -0.01, 0.005, 0.004, 0.0, -0.003]))
    hist = []
    T = oracle.register_rigid(p.model, None, p.obs, None, feat=3, residual="pt2pt", sigma=p.sigma,
                              w=p.w, iters=p.iters, T0=T0, lattice=lat, history=hist)
    assert all(h["stats"][2] > 0 for h in hist)
    err0 = oracle.alignment_error(T0, p.T_gt, p.model)
    err = oracle.alignment_error(T, p.T_gt, p.model)
    assert err < 0.25 * err0 and err < 0.005


def test_depth_frame_pt2pl_converges_from_near_start():
    p = synth.depth_pair(1, width=160, height=120, f=131.25)
    T0 = p.T_gt @ oracle.se3_exp(np.array([0.004, 0.003, -0.002, 0.005, -0.004, 0.003]))
    T = oracle.register_rigid(p.model, p.model_n, p.obs, p.obs_n, feat=6, residual="pt2pl", sigma=p.sigma,
                              sigma_n=p.sigma_n, w=p.w, iters=20, T0=T0)
    err0 = oracle.alignment_error(T0, p.T_gt, p.model)
    err = oracle.alignment_error(T, p.T_gt, p.model)
    assert err < 0.5 * err0
