"""Pins of the oracle's articulated kinematics (Sec. 5.1, Eq. 19-20, Alg. 1)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import articulated as art


def _tree(p):
    t = p.extra["tree"]
    return art.Tree(t.parent, t.dof_offset, t.origin, t.axis)


def test_forward_kinematics_matches_independent_posing():
    p = synth.articulated_pair(1, m=3000)
    tree = _tree(p)
    bo = p.extra["body_offsets"]
    for theta in (p.extra["theta_gt"], p.extra["theta0"], np.zeros(tree.n_dof)):
        x = art.pose_points(tree, theta, p.model, bo)
        Rs, ts = synth._pose_bodies(p.extra["tree"], theta)
        ref = np.concatenate([p.model[bo[b]:bo[b + 1]].astype(np.float64) @ Rs[b].T + ts[b]
                              for b in range(tree.n_bodies)])
        np.testing.assert_allclose(x, ref, atol=1e-14)


def test_spatial_jacobian_matches_finite_differences():
    """Column k of dzeta_b/dtheta is the left twist of T_b for a unit change of theta_k."""
    p = synth.articulated_pair(2, m=1000)
    tree = _tree(p)
    th = p.extra["theta_gt"]
    J = art.spatial_jacobians(tree, th)
    T0, _, _ = art.forward_kinematics(tree, th)
    h = 1e-6
    for k in range(tree.n_dof):
        dp, dm = th.copy(), th.copy()
        dp[k] += h
        dm[k] -= h
        Tp, _, _ = art.forward_kinematics(tree, dp)
        Tm, _, _ = art.forward_kinematics(tree, dm)
        for b in range(tree.n_bodies):
            dT = (Tp[b] - Tm[b]) / (2 * h) @ np.linalg.inv(T0[b])     # = [[w]x, v; 0, 0]
            w = np.array([dT[2, 1], dT[0, 2], dT[1, 0]])
            v = dT[:3, 3]
            np.testing.assert_allclose(J[b, :3, k], w, atol=1e-7)
            np.testing.assert_allclose(J[b, 3:, k], v, atol=1e-7)


@pytest.mark.parametrize("residual", ["pt2pt", "pt2pl"])
def test_alg1_equals_direct_assembly(residual):
    """Alg. 1 (per-body J^T J, then J_sp^T (.) J_sp) is an identity of the direct parameterisation."""
    p = synth.articulated_pair(3, m=4000)
    tree = _tree(p)
    bo = p.extra["body_offsets"]
    th = p.extra["theta0"]
    rng = np.random.default_rng(0)
    x = art.pose_points(tree, th, p.model, bo)
    M = len(x)
    m0 = rng.uniform(0.0, 2.0, M)
    m0[rng.uniform(size=M) < 0.1] = 0
    m1 = (x + rng.normal(scale=0.003, size=x.shape)) * m0[:, None]
    ns = rng.normal(size=(M, 3)) * m0[:, None]
    A1, b1 = art.normal_equations_alg1(tree, th, x, bo, m0, m1, ns, 0.2, 0.01, residual)
    A2, b2 = art.normal_equations_direct(tree, th, x, bo, m0, m1, ns, 0.2, 0.01, residual)
    np.testing.assert_allclose(A1, A2, rtol=0, atol=1e-10 * np.abs(A2).max())
    np.testing.assert_allclose(b1, b2, rtol=0, atol=1e-10 * np.abs(b2).max())
    assert np.linalg.matrix_rank(A1) == tree.n_dof


def separated_articulated(seed, sigma=0.0015, spacing=4.0):
    """A small noise-free articulated pair thinned so posed points are >= spacing * sigma apart."""
    p = synth.articulated_pair(seed, n_bodies=8, n_dof=12, m=900, noise=0.0, occlusion=0.0, sigma=sigma,
                               start_perturb=0.0005)
    tree = _tree(p)
    bo = p.extra["body_offsets"]
    y = art.pose_points(tree, p.extra["theta_gt"], p.model, bo)
    keep = []
    for i in range(len(y)):
        if not keep or np.min(np.linalg.norm(y[keep] - y[i], axis=1)) >= spacing * sigma:
            keep.append(i)
    keep = np.array(keep)
    body = np.searchsorted(bo, np.arange(len(y)), side="right") - 1
    counts = np.bincount(body[keep], minlength=tree.n_bodies)
    p.extra["body_offsets"] = np.concatenate([[0], np.cumsum(counts)])
    p.model, p.model_n = p.model[keep], p.model_n[keep]
    T, _, _ = art.forward_kinematics(tree, p.extra["theta_gt"])
    nb = p.extra["body_offsets"]
    p.obs = art.pose_points(tree, p.extra["theta_gt"], p.model, nb).astype(np.float32)
    p.obs_n = np.concatenate([p.model_n[nb[b]:nb[b + 1]].astype(np.float64) @ T[b, :3, :3].T
                              for b in range(tree.n_bodies)]).astype(np.float32)
    return p, tree


def test_articulated_exact_recovery():
    p, tree = separated_articulated(4)
    bo = p.extra["body_offsets"]
    assert len(p.model) > 150
    # separation: no two points share a lattice vertex at the ground truth or the start
    k = oracle.scale_factors(oracle.feature_sigmas(6, p.sigma, p.sigma_n))
    for th in (p.extra["theta_gt"], p.extra["theta0"]):
        x = art.pose_points(tree, th, p.model, bo).astype(np.float32)
        T, _, _ = art.forward_kinematics(tree, th)
        n = np.concatenate([p.model_n[bo[b]:bo[b + 1]].astype(np.float64) @ T[b, :3, :3].T
                            for b in range(tree.n_bodies)]).astype(np.float32)
        K = oracle.brute_force_lattice_sum(oracle.features(p.obs, p.obs_n, 6), np.eye(len(p.obs)),
                                           oracle.features(x, n, 6), k)
        assert np.all(K - np.diag(np.diag(K)) == 0)
    th = art.register_articulated(tree, p.model, p.model_n, bo, p.obs, p.obs_n, feat=6, residual="pt2pl",
                                  sigma=p.sigma, sigma_n=p.sigma_n, c=0.0, iters=10, theta0=p.extra["theta0"])
    assert np.abs(th - p.extra["theta_gt"]).max() < 1e-6
    assert np.abs(p.extra["theta0"] - p.extra["theta_gt"]).max() > 1e-4


def test_dofs_of_a_body_without_points_are_held():
    """The last body is a leaf; with none of its points in the model its DOFs move nothing.  They
    stay at their start values and the other DOFs follow exactly the registration of the tree
    without that body."""
    p, tree = separated_articulated(4)
    bo = p.extra["body_offsets"]
    B = tree.n_bodies
    assert not np.any(tree.parent == B - 1)
    nd = int(tree.dof_offset[B - 1])
    keep = slice(0, int(bo[B - 1]))
    bo_full = np.concatenate([bo[:B], [bo[B - 1]]])           # last body: 0 points
    th0 = p.extra["theta0"]
    kw = dict(feat=6, residual="pt2pl", sigma=p.sigma, sigma_n=p.sigma_n, c=0.0, iters=5)
    th_full = art.register_articulated(tree, p.model[keep], p.model_n[keep], bo_full, p.obs, p.obs_n,
                                       theta0=th0, **kw)
    sub = art.Tree(tree.parent[:B - 1], tree.dof_offset[:B], tree.origin[:B - 1], tree.axis[:nd])
    th_sub = art.register_articulated(sub, p.model[keep], p.model_n[keep], bo[:B], p.obs, p.obs_n,
                                      theta0=th0[:nd], **kw)
    np.testing.assert_array_equal(th_full[nd:], th0[nd:])
    np.testing.assert_allclose(th_full[:nd], th_sub, rtol=0, atol=1e-12)
