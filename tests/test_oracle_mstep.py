"""Pins of the oracle's M-step (Sec. 3.1 Eq. 7, Sec. 3.3 Eq. 10, Sec. 5 Eq. 15-18).

* the twist Jacobian against finite differences of the exponential update,
* the SE(3) exponential against scipy's matrix exponential,
* Gauss-Newton with fixed targets against the closed-form weighted Procrustes
  (Kabsch/Umeyama SVD),
* point-to-plane: one step recovers a pure translation exactly.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle


def twist_matrix(z):
    W = np.zeros((4, 4))
    W[:3, :3] = oracle.skew(z[:3])
    W[:3, 3] = z[3:]
    return W


def test_exp_matches_matrix_exponential():
    rng = np.random.default_rng(0)
    for scale in (1e-7, 1e-5, 1e-4 * 0.999, 1e-4 * 1.001, 1e-2, 0.3, 2.0, 3.1):
        for _ in range(20):
            z = rng.normal(size=6)
            z[:3] *= scale / np.linalg.norm(z[:3])
            T = oracle.se3_exp(z)
            ref = scipy.linalg.expm(twist_matrix(z))
            np.testing.assert_allclose(T, ref, atol=1e-12)
            R = T[:3, :3]
            np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)


def test_exp_is_continuous_across_series_switch():
    z = np.array([1.0, -2.0, 0.5, 0.1, 0.2, 0.3])
    z1, z2 = z.copy(), z.copy()
    z1[:3] *= (1e-4 * (1 - 1e-9)) / np.linalg.norm(z[:3])
    z2[:3] *= (1e-4 * (1 + 1e-9)) / np.linalg.norm(z[:3])
    assert np.abs(oracle.se3_exp(z1) - oracle.se3_exp(z2)).max() < 1e-12


@pytest.mark.parametrize("residual", ["pt2pt", "pt2pl"])
def test_jacobian_matches_finite_differences(residual):
    """d r / d zeta for x(zeta) = Exp(zeta) x at zeta = 0, with M0/M1/N held fixed."""
    rng = np.random.default_rng(1)
    M = 50
    x = rng.normal(size=(M, 3))
    m0 = rng.uniform(0.5, 2.0, size=M)
    m1 = (x + rng.normal(scale=0.1, size=(M, 3))) * m0[:, None]
    ns = rng.normal(size=(M, 3)) * m0[:, None]
    sigma = 0.07
    _, r0, J, _ = oracle.residuals_and_jacobians(x, m0, m1, ns, 0.3, sigma, residual)
    h = 1e-6
    for p in range(6):
        dz = np.zeros(6)
        dz[p] = h
        xp = x @ oracle.se3_exp(dz)[:3, :3].T + oracle.se3_exp(dz)[:3, 3]
        xm = x @ oracle.se3_exp(-dz)[:3, :3].T + oracle.se3_exp(-dz)[:3, 3]
        _, rp, _, _ = oracle.residuals_and_jacobians(xp, m0, m1, ns, 0.3, sigma, residual)
        _, rm, _, _ = oracle.residuals_and_jacobians(xm, m0, m1, ns, 0.3, sigma, residual)
        fd = (rp - rm) / (2 * h)
        np.testing.assert_allclose(J[:, :, p], fd, atol=1e-6 * np.abs(fd).max() + 1e-8)


def weighted_kabsch(src, dst, w):
    """Closed-form weighted rigid fit of src onto dst (Umeyama without scale)."""
    mu_s = (w[:, None] * src).sum(0) / w.sum()
    mu_d = (w[:, None] * dst).sum(0) / w.sum()
    H = ((src - mu_s) * w[:, None]).T @ (dst - mu_d)
    U, _, Vt = np.linalg.svd(H)
    S = np.eye(3)
    S[2, 2] = np.sign(np.linalg.det(Vt.T @ U.T))
    R = Vt.T @ S @ U.T
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = mu_d - R @ mu_s
    return T


def test_gauss_newton_with_fixed_targets_converges_to_weighted_procrustes():
    rng = np.random.default_rng(2)
    M = 400
    x_ref = rng.normal(size=(M, 3))
    tgt = x_ref @ oracle.se3_exp(np.array([0.3, -0.2, 0.1, 0.5, -0.1, 0.2]))[:3, :3].T + np.array([0.3, 0.1, -0.2])
    tgt += rng.normal(scale=0.05, size=tgt.shape)
    m0 = rng.uniform(0.2, 3.0, size=M)
    c = 0.7
    w = m0 / (m0 + c)
    m1 = tgt * m0[:, None]
    T = np.eye(4)
    for _ in range(30):
        x = x_ref @ T[:3, :3].T + T[:3, 3]
        A, b, _ = oracle.normal_equations(x, m0, m1, None, c, 0.05, "pt2pt")
        T = oracle.se3_exp(oracle.gn_step(A, b)) @ T
    ref = weighted_kabsch(x_ref, tgt, w)
    np.testing.assert_allclose(T, ref, atol=1e-10)


def test_point_to_plane_recovers_translation_in_one_step():
    rng = np.random.default_rng(3)
    M = 300
    y = rng.normal(size=(M, 3))
    n = rng.normal(size=(M, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    t = np.array([0.02, -0.03, 0.01])
    x = y - t          # model = observation shifted; exact correspondences with exact normals
    m0 = np.ones(M)
    A, b, _ = oracle.normal_equations(x, m0, y * m0[:, None], n * m0[:, None], 0.0, 0.01, "pt2pl")
    dz = oracle.gn_step(A, b)
    np.testing.assert_allclose(dz[:3], 0.0, atol=1e-12)
    np.testing.assert_allclose(dz[3:], t, atol=1e-12)


def test_weights_support_and_stats():
    x = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    m0 = np.array([2.0, 0.0, 1.0])
    m1 = np.array([[0.2, 0, 0], [5, 5, 5], [0, 1.1, 0]])
    w, r, J, sup = oracle.residuals_and_jacobians(x, m0, m1, None, 1.0, 0.5, "pt2pt")
    np.testing.assert_allclose(w, [2 / 3, 0.0, 0.5])
    assert sup.tolist() == [True, False, True]
    np.testing.assert_allclose(r[0], [-0.2, 0, 0])         # (x - M1/M0) / sigma
    np.testing.assert_allclose(r[2], [0, -0.2, 0])
    assert np.all(r[1] == 0) and np.all(J[1] == 0)
    A, b, st = oracle.normal_equations(x, m0, m1, None, 1.0, 0.5, "pt2pt")
    np.testing.assert_allclose(st, [2 / 3 + 0.5, 2 / 3 * 0.04 + 0.5 * 0.04, 2, 3.0])


def test_degenerate_system_raises():
    with pytest.raises(oracle.Degenerate):
        oracle.gn_step(np.zeros((6, 6)), np.zeros(6))


def _plane_system(normals_of_planes, seed=0, n=300):
    """Point-to-plane normal equations of points on the given planes through the origin, each point
    with its plane's normal and a unit weight (Eq. 10 with the rigid Jacobian of Sec. 5)."""
    rng = np.random.default_rng(seed)
    A = np.zeros((6, 6))
    for nrm in normals_of_planes:
        nrm = np.asarray(nrm, float) / np.linalg.norm(nrm)
        u = np.cross(nrm, [1.0, 0.3, 0.1]); u /= np.linalg.norm(u)
        v = np.cross(nrm, u)
        x = rng.uniform(-1, 1, (n, 1)) * u + rng.uniform(-1, 1, (n, 1)) * v
        J = oracle.point_jacobian(x)                      # (n, 3, 6)
        row = np.einsum("k,ikp->ip", nrm, J)              # n^T J
        A += row.T @ row
    return A


def test_planar_point_to_plane_system_has_rank_three_and_is_refused():
    # one plane constrains the translation along its normal and the two rotations about axes in it:
    # rank 3, whatever the rounding of the sums
    A = _plane_system([[0.2, -0.1, 1.0]])
    ev = np.linalg.eigvalsh(A)
    assert (np.abs(ev[:3]) < 1e-9 * ev[-1]).all() and (ev[3:] > 1e-3 * ev[-1]).all()
    b = np.ones(6)
    with pytest.raises(oracle.Degenerate):
        oracle.gn_step(A, b, oracle.RIGID_PIVOT_TOL)
    # binary32-sized perturbations can make it numerically positive definite; the relative pivot rule
    # still refuses it, where the bare Cholesky would not
    rng = np.random.default_rng(1)
    for _ in range(20):
        E = rng.normal(size=(6, 6)) * 3e-6 * np.abs(A).max()
        Ap = A + E @ E.T / 6 + np.eye(6) * 1e-7 * np.abs(A).max()
        oracle.gn_step(Ap, b)                                  # no error without the rule
        with pytest.raises(oracle.Degenerate):
            oracle.gn_step(Ap, b, oracle.RIGID_PIVOT_TOL)


def test_three_planes_pass_the_pivot_rule():
    A = _plane_system([[1, 0, 0.1], [0, 1, 0.2], [0.1, 0.1, 1]])
    L = np.linalg.cholesky(A)
    assert (np.diag(L) ** 2 / np.diag(A)).min() > 100 * oracle.RIGID_PIVOT_TOL
    x = oracle.gn_step(A, np.ones(6), oracle.RIGID_PIVOT_TOL)
    np.testing.assert_allclose(A @ x, -np.ones(6), rtol=0, atol=1e-9 * np.abs(A).max())


def test_pivot_rule_threshold_on_designed_systems():
    # A = L L^T with unit diagonal and one chosen relative pivot L_jj^2 / A_jj at the last position:
    # 1e-3 passes (the step solves A x = -b), 1e-5 is refused, as is 1e-4 itself (at or below the rule)
    rng = np.random.default_rng(3)
    for rel, ok in ((1e-3, True), (2e-4, True), (1e-4, False), (1e-5, False)):
        for _ in range(5):
            u = rng.normal(size=5)
            u /= np.linalg.norm(u)
            L = np.zeros((6, 6))
            L[:5, :5] = np.eye(5)
            L[5, :5] = u * math.sqrt(1.0 - rel)
            L[5, 5] = math.sqrt(rel)
            A = L @ L.T
            assert np.isclose(np.linalg.cholesky(A)[5, 5] ** 2 / A[5, 5], rel, rtol=1e-9)
            b = rng.normal(size=6)
            if ok:
                x = oracle.gn_step(A, b, oracle.RIGID_PIVOT_TOL)
                np.testing.assert_allclose(A @ x, -b, atol=1e-9)
            else:
                with pytest.raises(oracle.Degenerate):
                    oracle.gn_step(A, b, oracle.RIGID_PIVOT_TOL)
                oracle.gn_step(A, b)          # positive definite: only the rule refuses it


def test_outlier_constant_zero_cases():
    assert oracle.outlier_constant(0.0, 10, 10, (1, 1, 1)) == 0.0
    assert oracle.outlier_constant(0.3, 10, 0, (1, 1, 1)) == 0.0
    # linear in N/M and in every width; w/(1-w) in w
    c = oracle.outlier_constant(0.5, 200, 100, (0.1, 0.2, 0.3))
    assert math.isclose(oracle.outlier_constant(0.5, 400, 100, (0.1, 0.2, 0.3)), 2 * c, rel_tol=1e-14)
    assert math.isclose(oracle.outlier_constant(0.5, 200, 100, (0.2, 0.2, 0.3)), 2 * c, rel_tol=1e-14)
    assert math.isclose(oracle.outlier_constant(0.75, 200, 100, (0.1, 0.2, 0.3)), 3 * c, rel_tol=1e-14)
