"""Pins of the oracle's node-graph kinematics (Sec. 5.2, Eq. 21)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import nodegraph as ng


def _graph(p):
    e = p.extra
    return ng.Graph(e["nodes"], e["skin_idx"], e["skin_w"], e["edges"])


def _T(R, t):
    T = np.zeros((len(R), 4, 4))
    T[:, :3, :3] = R
    T[:, :3, 3] = t
    T[:, 3, 3] = 1.0
    return T


def test_dual_quaternion_round_trip_and_independent_blend():
    p = synth.nodegraph_pair(1, m=4000, n_nodes=64)
    g = _graph(p)
    T = _T(p.extra["node_R"], p.extra["node_t"])
    for k in range(5):
        qr, qd = ng.dual_quat(T[k])
        np.testing.assert_allclose(ng.matrix_from_dual_quat(qr, qd), T[k], atol=1e-14)
    x, n = ng.warp(T, g, p.model, p.model_n)
    R, t = synth._dq_blend(p.extra["node_R"], p.extra["node_t"], g.skin_idx, g.skin_w)
    np.testing.assert_allclose(x, np.einsum("ijk,ik->ij", R, p.model.astype(np.float64)) + t, atol=1e-13)


def test_blend_of_equal_nodes_is_that_transform():
    p = synth.nodegraph_pair(2, m=2000, n_nodes=32)
    g = _graph(p)
    Tr = synth.random_motion(np.random.default_rng(0), 0.7, 0.3)
    Ti = ng.blend_transforms(np.repeat(Tr[None], 32, 0), g)
    np.testing.assert_allclose(Ti, np.broadcast_to(Tr, Ti.shape), atol=1e-14)


def test_point_twist_is_the_blend_of_node_twists_at_agreement():
    """d x_i / d zeta_k = w_ki [-[x]_x, I] where all nodes agree (the Jacobian reading)."""
    p = synth.nodegraph_pair(3, m=300, n_nodes=16)
    g = _graph(p)
    K = 16
    T = np.repeat(synth.random_motion(np.random.default_rng(1), 0.3, 0.1)[None], K, 0)
    x0, _ = ng.warp(T, g, p.model)
    h = 1e-6
    rng = np.random.default_rng(2)
    for _ in range(6):
        k = int(rng.integers(0, K))
        z = rng.normal(size=6)
        Tp, Tm = T.copy(), T.copy()
        Tp[k] = oracle.se3_exp(h * z) @ T[k]
        Tm[k] = oracle.se3_exp(-h * z) @ T[k]
        dx = (ng.warp(Tp, g, p.model)[0] - ng.warp(Tm, g, p.model)[0]) / (2 * h)
        wk = np.where(g.skin_idx == k, g.skin_w, 0.0).sum(1)
        ref = wk[:, None] * (oracle.point_jacobian(x0) @ z)
        np.testing.assert_allclose(dx, ref, atol=1e-6)


def test_common_twist_reduces_to_rigid_normal_equations():
    """Summing the node blocks over nodes (all node twists equal) gives the rigid A and b; the
    regulariser vanishes for equal node transforms."""
    p = synth.nodegraph_pair(4, m=3000, n_nodes=32)
    g = _graph(p)
    K = 32
    rng = np.random.default_rng(3)
    T = np.repeat(synth.random_motion(rng, 0.2, 0.05)[None], K, 0)
    x, _ = ng.warp(T, g, p.model)
    m0 = rng.uniform(0, 2, len(x))
    m1 = (x + rng.normal(scale=0.01, size=x.shape)) * m0[:, None]
    A, b = ng.node_blocks(g, T, x, m0, m1, None, 0.3, 0.02, "pt2pt", lam=2.0)
    Ar, br, _ = oracle.normal_equations(x, m0, m1, None, 0.3, 0.02, "pt2pt")
    A4 = A.reshape(K, 6, K, 6)
    np.testing.assert_allclose(A4.sum(axis=(0, 2)), Ar, rtol=1e-10, atol=1e-9 * np.abs(Ar).max())
    np.testing.assert_allclose(b.reshape(K, 6).sum(0), br, rtol=1e-10, atol=1e-9 * np.abs(br).max())
    np.testing.assert_allclose(A, A.T, atol=1e-9 * np.abs(A).max())


def test_nodegraph_recovers_a_rigid_motion_exactly():
    """Separated noise-free points under one rigid motion of all nodes: the data residual and the
    regulariser both vanish at the ground truth, and Gauss-Newton lands on it."""
    p = synth.separated_pair(5, 500, sigma=0.01, feat=3)
    T_gt = p.T_gt
    rng = np.random.default_rng(4)
    K = 12
    nodes = p.model[rng.choice(len(p.model), K, replace=False)].astype(np.float64)
    d = np.linalg.norm(p.model[:, None, :] - nodes[None], axis=-1)
    idx = np.argsort(d, 1)[:, :4]
    dd = np.take_along_axis(d, idx, 1)
    w = np.exp(-dd ** 2 / (2 * 0.1 ** 2)) + 1e-12
    w /= w.sum(1, keepdims=True)
    ie = np.argsort(np.linalg.norm(nodes[:, None] - nodes[None], axis=-1), 1)[:, 1:5]   # 4 nearest other nodes
    edges = np.array([(j, k) for j in range(K) for k in ie[j]])
    g = ng.Graph(nodes, idx.astype(np.int32), w, edges)
    T0 = np.repeat(p.extra["T0"][None], K, 0)
    T = ng.register_nodegraph(g, p.model, None, p.obs, None, sigma=p.sigma, c=0.0, lam=1.0, iters=12, T0=T0)
    for k in range(K):
        np.testing.assert_allclose(T[k], T_gt, atol=1e-6)


def _regulariser_energy(g, T, lam, sigma):
    """lam sum over directed edges (j, k) of |(T_j p_k - T_k p_k) / sigma|^2 (Eq. 21's regulariser)."""
    E = 0.0
    for j, k in g.edges:
        pk = g.nodes[k]
        e = (T[j][:3, :3] @ pk + T[j][:3, 3] - T[k][:3, :3] @ pk - T[k][:3, 3]) / sigma
        E += lam * float(e @ e)
    return E


def _spread_nodes(seed, K=10):
    """A small graph and node transforms that all differ (no agreement anywhere)."""
    p = synth.nodegraph_pair(seed, m=400, n_nodes=K)
    g = _graph(p)
    rng = np.random.default_rng(seed + 100)
    T = np.stack([synth.random_motion(rng, 0.4, 0.1) for _ in range(K)])
    return p, g, T


def _regulariser_blocks(g, T, lam, sigma):
    """node_blocks with no supported point: only the regulariser's A and b remain."""
    x = np.zeros((3, 3))
    z = np.zeros(3)
    g0 = ng.Graph(g.nodes, np.zeros((3, 4), np.int32), np.full((3, 4), 0.25), g.edges)
    return ng.node_blocks(g0, T, x, z, np.zeros((3, 3)), None, 1.0, sigma, "pt2pt", lam)


def test_regulariser_b_is_half_the_energy_gradient_away_from_agreement():
    """b of the linearised regulariser is J^T e: half the gradient of the energy in the node twists
    (left-multiplied, T_k <- Exp(zeta_k) T_k), checked by central differences of the energy at unequal
    node transforms.  A flipped residual sign or b term, or a Jacobian taken at the other end of an
    edge, fails it."""
    lam, sigma = 1.7, 0.02
    p, g, T = _spread_nodes(6)
    K = len(g.nodes)
    _, b = _regulariser_blocks(g, T, lam, sigma)
    h = 1e-6
    grad = np.zeros(6 * K)
    for k in range(K):
        for q in range(6):
            z = np.zeros(6)
            z[q] = h
            Tp, Tm = T.copy(), T.copy()
            Tp[k] = oracle.se3_exp(z) @ T[k]
            Tm[k] = oracle.se3_exp(-z) @ T[k]
            grad[6 * k + q] = (_regulariser_energy(g, Tp, lam, sigma) - _regulariser_energy(g, Tm, lam, sigma)) / (2 * h)
    assert np.abs(b).max() > 1.0
    np.testing.assert_allclose(b, 0.5 * grad, rtol=1e-6, atol=1e-6 * np.abs(grad).max())


def test_regulariser_gauss_newton_matrix_from_finite_difference_jacobians():
    """A of the regulariser is lam sum J^T J with J the derivative of each edge residual in the twists of
    both end nodes, evaluated at unequal transforms by central differences of the residual itself."""
    lam, sigma = 0.6, 0.03
    p, g, T = _spread_nodes(7)
    K = len(g.nodes)
    A, _ = _regulariser_blocks(g, T, lam, sigma)
    h = 1e-6
    Afd = np.zeros((6 * K, 6 * K))
    for j, k in g.edges:
        pk = g.nodes[k]

        def res(Tj, Tk):
            return (Tj[:3, :3] @ pk + Tj[:3, 3] - Tk[:3, :3] @ pk - Tk[:3, 3]) / sigma
        J = np.zeros((3, 6 * K))
        for node in (j, k):
            for q in range(6):
                z = np.zeros(6)
                z[q] = h
                Tp, Tm = T.copy(), T.copy()
                Tp[node] = oracle.se3_exp(z) @ T[node]
                Tm[node] = oracle.se3_exp(-z) @ T[node]
                J[:, 6 * node + q] += (res(Tp[j], Tp[k]) - res(Tm[j], Tm[k])) / (2 * h)
        Afd += lam * J.T @ J
    np.testing.assert_allclose(A, Afd, rtol=1e-6, atol=1e-6 * np.abs(Afd).max())


def test_regulariser_step_reduces_its_energy():
    """One Gauss-Newton step of the regulariser alone (anchored by a tiny ridge) lowers the energy."""
    lam, sigma = 1.0, 0.02
    p, g, T = _spread_nodes(8)
    K = len(g.nodes)
    A, b = _regulariser_blocks(g, T, lam, sigma)
    dz = np.linalg.solve(A + 1e-9 * np.abs(A).max() * np.eye(6 * K), -b).reshape(K, 6)
    T1 = np.stack([oracle.se3_exp(0.5 * dz[k]) @ T[k] for k in range(K)])
    assert _regulariser_energy(g, T1, lam, sigma) < 0.5 * _regulariser_energy(g, T, lam, sigma)
