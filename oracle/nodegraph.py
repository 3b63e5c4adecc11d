"""Node-graph deformable kinematics for the oracle (Sec. 5.2, Eq. 21).  TEST INFRASTRUCTURE ONLY.

A node graph is a set of nodes {p_j, T_j}; each model point is skinned to K
nearest nodes with fixed weights w_ki, and moves by the normalised dual-
quaternion blend of their transforms (Eq. 21, dual quaternions of the cited
Kavan et al. blending).

Readings (the supplement that details the node-graph A-matrix is not available):
* skin weights w_ki proportional to exp(-|x_ref - p_k|^2 / (2 r^2)) over the 4
  nearest nodes, normalised, r = mean nearest-node spacing;
* the twist of point i is the blend of node twists, d zeta_i / d zeta_k = w_ki I6
  (exact where the blended nodes agree, e.g. at the start from identity);
  so the data blocks are A_kl += w_ki w_li J_i^T J_i and b_k += w_ki J_i^T r_i;
* regulariser lambda sum over directed 8-NN edges (j, k) of |(T_j p_k - T_k p_k) / sigma|^2,
  linearised with the twist Jacobians of both ends;
* nodes are updated by T_k <- Exp(dzeta_k) T_k.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import residuals_and_jacobians, se3_exp, gn_step, estep, build_observation_lattice, outlier_constant, skew, \
    feature_sigmas


@dataclasses.dataclass
class Graph:
    nodes: np.ndarray      # (K, 3) reference node positions
    skin_idx: np.ndarray   # (M, 4) node indices per point
    skin_w: np.ndarray     # (M, 4) weights (rows sum to 1)
    edges: np.ndarray      # (E, 2) directed regulariser edges (j, k)


# --- dual quaternions (Hamilton product, w first) ----------------------------------
def qmul(a, b):
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], -1)


def quat_from_matrix(R):
    """Unit quaternion (w, x, y, z) of a rotation matrix (largest-pivot method)."""
    R = np.asarray(R, dtype=np.float64)
    tr = np.trace(R)
    if tr > 0:
        s = np.sqrt(tr + 1.0) * 2
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif R[1, 1] > R[2, 2]:
        s = np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.asarray(q)
    return q / np.linalg.norm(q)


def dual_quat(T):
    """(real, dual) parts of the unit dual quaternion of a rigid transform: d = t q / 2."""
    qr = quat_from_matrix(T[:3, :3])
    tq = np.concatenate([[0.0], T[:3, 3]])
    return qr, 0.5 * qmul(tq, qr)


def matrix_from_dual_quat(qr, qd):
    """Rigid transform of a unit dual quaternion: R from qr, t = 2 qd conj(qr)."""
    w, x, y, z = qr
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    conj = qr * np.array([1.0, -1.0, -1.0, -1.0])
    t = 2.0 * qmul(qd, conj)[1:]
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def blend_transforms(T_nodes, graph: Graph):
    """Per-point rigid transforms (M, 4, 4) by normalised dual-quaternion blending (Eq. 21).
    Quaternion signs are aligned with the point's first node (shortest-path blending)."""
    dq = [dual_quat(T) for T in T_nodes]
    qr = np.stack([a for a, _ in dq])
    qd = np.stack([b for _, b in dq])
    idx = graph.skin_idx
    w = graph.skin_w
    ref = qr[idx[:, 0]]                                            # (M, 4)
    sgn = np.where(np.einsum("mj,mkj->mk", ref, qr[idx]) >= 0, 1.0, -1.0)
    br = np.einsum("mk,mkj->mj", sgn * w, qr[idx])
    bd = np.einsum("mk,mkj->mj", sgn * w, qd[idx])
    nrm = np.linalg.norm(br, axis=1, keepdims=True)
    br, bd = br / nrm, bd / nrm
    wq, xq, yq, zq = br[:, 0], br[:, 1], br[:, 2], br[:, 3]
    M = len(idx)
    out = np.zeros((M, 4, 4))
    out[:, 0, 0] = 1 - 2 * (yq * yq + zq * zq)
    out[:, 0, 1] = 2 * (xq * yq - wq * zq)
    out[:, 0, 2] = 2 * (xq * zq + wq * yq)
    out[:, 1, 0] = 2 * (xq * yq + wq * zq)
    out[:, 1, 1] = 1 - 2 * (xq * xq + zq * zq)
    out[:, 1, 2] = 2 * (yq * zq - wq * xq)
    out[:, 2, 0] = 2 * (xq * zq - wq * yq)
    out[:, 2, 1] = 2 * (yq * zq + wq * xq)
    out[:, 2, 2] = 1 - 2 * (xq * xq + yq * yq)
    out[:, :3, 3] = 2.0 * qmul(bd, br * np.array([1.0, -1.0, -1.0, -1.0]))[:, 1:]
    out[:, 3, 3] = 1.0
    return out


def warp(T_nodes, graph: Graph, x_ref, n_ref=None):
    """Blended point positions (and normals) in float64."""
    Ti = blend_transforms(T_nodes, graph)
    x = np.einsum("ijk,ik->ij", Ti[:, :3, :3], np.asarray(x_ref, dtype=np.float64)) + Ti[:, :3, 3]
    n = None
    if n_ref is not None:
        n = np.einsum("ijk,ik->ij", Ti[:, :3, :3], np.asarray(n_ref, dtype=np.float64))
    return x, n


def node_blocks(graph: Graph, T_nodes, x, m0, m1, ns, c, sigma, residual, lam):
    """Dense (6K x 6K) normal equations of the node twists: data blocks w_ki w_li J^T J and the
    linearised edge regulariser."""
    from . import per_point_jtj
    K = len(graph.nodes)
    A = np.zeros((6 * K, 6 * K))
    b = np.zeros(6 * K)
    JtJ, Jtr = per_point_jtj(x, m0, m1, ns, c, sigma, residual)
    for a in range(graph.skin_idx.shape[1]):
        ka = graph.skin_idx[:, a]
        wa = graph.skin_w[:, a]
        np.add.at(b.reshape(K, 6), ka, wa[:, None] * Jtr)
        for c2 in range(graph.skin_idx.shape[1]):
            kb = graph.skin_idx[:, c2]
            wb = graph.skin_w[:, c2]
            blk = (wa * wb)[:, None, None] * JtJ
            A4 = A.reshape(K, 6, K, 6)
            np.add.at(A4, (ka, slice(None), kb, slice(None)), blk)
    if lam > 0:
        for j, k in graph.edges:
            pk = graph.nodes[k]
            xj = T_nodes[j][:3, :3] @ pk + T_nodes[j][:3, 3]
            xk = T_nodes[k][:3, :3] @ pk + T_nodes[k][:3, 3]
            e = (xj - xk) / sigma
            Jj = np.concatenate([-skew(xj), np.eye(3)], 1) / sigma
            Jk = -np.concatenate([-skew(xk), np.eye(3)], 1) / sigma
            sj, sk = slice(6 * j, 6 * j + 6), slice(6 * k, 6 * k + 6)
            A[sj, sj] += lam * Jj.T @ Jj
            A[sk, sk] += lam * Jk.T @ Jk
            A[sj, sk] += lam * Jj.T @ Jk
            A[sk, sj] += lam * Jk.T @ Jj
            b[sj] += lam * Jj.T @ e
            b[sk] += lam * Jk.T @ e
    return A, b


def register_nodegraph(graph: Graph, x_ref, n_ref, obs, obs_n, *, feat=3, residual="pt2pt", sigma, sigma_n=0.5,
                       c=None, w=0.1, lam=1.0, iters=20, T0=None, history=None):
    """Node-graph FilterReg: lattice built once; per EM iteration warp (binary64, rounded to
    binary32 for the E-step), slice, node normal equations, dense Cholesky solve,
    T_k <- Exp(dzeta_k) T_k."""
    K = len(graph.nodes)
    T = np.repeat(np.eye(4)[None], K, 0) if T0 is None else np.array(T0, dtype=np.float64)
    if c is None:
        c = outlier_constant(w, len(obs), len(x_ref), feature_sigmas(feat, sigma, sigma_n))
    sig_m = float(np.mean(sigma))
    lat = build_observation_lattice(obs, obs_n, feat, residual, sigma, sigma_n)
    for _ in range(iters):
        x64, n64 = warp(T, graph, x_ref, n_ref if feat == 6 else None)
        x32 = x64.astype(np.float32)
        n32 = n64.astype(np.float32) if n64 is not None else None
        m0, m1, ns = estep(lat, x32, n32, feat, residual)
        A, b = node_blocks(graph, T, x32.astype(np.float64), m0, m1, ns, c, sig_m, residual, lam)
        dz = gn_step(A, b).reshape(K, 6)
        T = np.stack([se3_exp(dz[k]) @ T[k] for k in range(K)])
        if history is not None:
            history.append(dict(A=A, b=b, dz=dz, T=T.copy()))
    return T
