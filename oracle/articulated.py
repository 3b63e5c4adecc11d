"""Articulated kinematics for the oracle (Sec. 5.1, Eq. 19-20, Alg. 1).  TEST INFRASTRUCTURE ONLY.

Kinematic tree: bodies b = 0..B-1 with parent[b] < b (-1 = world).  Body b owns
the revolute DOFs [dof_offset[b], dof_offset[b+1]); its frame is

    T_b = T_parent(b) . Trans(o_b) . Rot(a_k0, theta_k0) . Rot(a_k1, theta_k1) ...

with the joint origin o_b in the parent frame and each axis a_k in the frame
left by the preceding rotations.  A model point on body b moves as
x = T_b(theta) x_ref (Eq. 15).

Twists use the convention of Eq. 16 (x_new = x + w x x + v).  A unit change of
DOF k rotates every descendant of its joint about the world axis w_k through
the world point q_k, i.e. the twist (w_k, q_k x w_k); these columns form the
spatial velocity Jacobian of each body (dzeta_b / dtheta).  Alg. 1 sums the
per-point J^T J of each body and then A = sum_b J_sp,b^T (J^TJ)_b J_sp,b.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import residuals_and_jacobians, se3_exp, gn_step, estep, pose_to_mat12, transform_f32, RIGID_PIVOT_TOL, \
    build_observation_lattice, outlier_constant, feature_sigmas


@dataclasses.dataclass
class Tree:
    parent: np.ndarray        # (B,) int
    dof_offset: np.ndarray    # (B+1,) int
    origin: np.ndarray        # (B, 3) joint origin in the parent frame
    axis: np.ndarray          # (n_dof, 3) unit axis in the frame before its rotation

    @property
    def n_bodies(self):
        return len(self.parent)

    @property
    def n_dof(self):
        return int(self.dof_offset[-1])


def _rot(axis, angle):
    z = np.zeros(6)
    z[:3] = np.asarray(axis, dtype=np.float64) * angle
    return se3_exp(z)


def forward_kinematics(tree: Tree, theta: np.ndarray):
    """Body frames T (B, 4, 4) and, per DOF, the world axis w_k (n_dof, 3) and point q_k (n_dof, 3)."""
    B = tree.n_bodies
    T = np.zeros((B, 4, 4))
    w = np.zeros((tree.n_dof, 3))
    q = np.zeros((tree.n_dof, 3))
    for b in range(B):
        P = np.eye(4) if tree.parent[b] < 0 else T[tree.parent[b]]
        F = P.copy()
        F[:3, 3] = P[:3, :3] @ tree.origin[b] + P[:3, 3]
        for k in range(tree.dof_offset[b], tree.dof_offset[b + 1]):
            w[k] = F[:3, :3] @ tree.axis[k]
            q[k] = F[:3, 3]
            F = F @ _rot(tree.axis[k], theta[k])
        T[b] = F
    return T, w, q


def ancestors_dofs(tree: Tree, b: int):
    """DOFs that move body b: its own and those of all its ancestors."""
    out = []
    while b >= 0:
        out.extend(range(tree.dof_offset[b], tree.dof_offset[b + 1]))
        b = tree.parent[b]
    return sorted(out)


def spatial_jacobians(tree: Tree, theta: np.ndarray) -> np.ndarray:
    """dzeta_b / dtheta (B, 6, n_dof): column k = (w_k, q_k x w_k) if DOF k moves body b."""
    _, w, q = forward_kinematics(tree, theta)
    J = np.zeros((tree.n_bodies, 6, tree.n_dof))
    for b in range(tree.n_bodies):
        for k in ancestors_dofs(tree, b):
            J[b, :3, k] = w[k]
            J[b, 3:, k] = np.cross(q[k], w[k])
    return J


def pose_points(tree: Tree, theta, x_ref, body_offsets):
    """x = T_b(theta) x_ref for points grouped by body (float64)."""
    T, _, _ = forward_kinematics(tree, theta)
    x = np.zeros((len(x_ref), 3))
    for b in range(tree.n_bodies):
        sl = slice(body_offsets[b], body_offsets[b + 1])
        x[sl] = np.asarray(x_ref[sl], dtype=np.float64) @ T[b, :3, :3].T + T[b, :3, 3]
    return x


def normal_equations_alg1(tree, theta, x, body_offsets, m0, m1, ns, c, sigma, residual):
    """Alg. 1: per-body sums of J^T J and J^T r, then A = sum_b J_sp^T (J^TJ)_b J_sp."""
    from . import per_point_jtj
    JtJ, Jtr = per_point_jtj(x, m0, m1, ns, c, sigma, residual)
    Jsp = spatial_jacobians(tree, theta)
    A = np.zeros((tree.n_dof, tree.n_dof))
    bvec = np.zeros(tree.n_dof)
    for b in range(tree.n_bodies):
        sl = slice(body_offsets[b], body_offsets[b + 1])
        Sb = JtJ[sl].sum(0)
        sb = Jtr[sl].sum(0)
        A += Jsp[b].T @ Sb @ Jsp[b]
        bvec += Jsp[b].T @ sb
    return A, bvec


def normal_equations_direct(tree, theta, x, body_offsets, m0, m1, ns, c, sigma, residual):
    """Direct parameterisation: dr/dtheta_k through dx/dtheta_k = w_k x (x - q_k), O(n_dof^2 M)."""
    w_, q_ = forward_kinematics(tree, theta)[1:]
    w, r, Jz, _ = residuals_and_jacobians(x, m0, m1, ns, c, sigma, residual)
    # dr/dx: undo the twist Jacobian's x-dependence by using its translation block (dr/dt = dr/dx)
    drdx = Jz[:, :, 3:]                                    # (M, k, 3)
    A = np.zeros((tree.n_dof, tree.n_dof))
    bvec = np.zeros(tree.n_dof)
    for b in range(tree.n_bodies):
        sl = slice(body_offsets[b], body_offsets[b + 1])
        dofs = ancestors_dofs(tree, b)
        dxdth = np.zeros((sl.stop - sl.start, 3, tree.n_dof))
        for k in dofs:
            dxdth[:, :, k] = np.cross(w_[k][None, :], x[sl] - q_[k][None, :])
        Jt = np.einsum("ikx,ixn->ikn", drdx[sl], dxdth)
        A += np.einsum("i,ikn,ikm->nm", w[sl], Jt, Jt)
        bvec += np.einsum("i,ikn,ik->n", w[sl], Jt, r[sl])
    return A, bvec


def hold_unsupported(A, b):
    """A DOF that moves no supported point has an all-zero row and column in A (Alg. 1 sums
    only supported points).  Reading: such a DOF is held, dtheta_k = 0, and the other DOFs are
    solved as if it were absent (its row/column replaced by the identity, b_k = 0)."""
    held = np.diag(A) == 0.0
    if not held.any():
        return A, b
    A = A.copy()
    A[held, :] = 0.0
    A[:, held] = 0.0
    A[held, held] = 1.0
    return A, np.where(held, 0.0, b)


def register_articulated(tree: Tree, x_ref, n_ref, body_offsets, obs, obs_n, *, feat, residual, sigma,
                         sigma_n=0.5, c=None, w=0.1, iters=15, theta0=None, history=None):
    """Articulated FilterReg: lattice built once, then per EM iteration slice at the pinned
    binary32 body transforms, Alg. 1 normal equations, theta += -A^-1 b."""
    theta = np.zeros(tree.n_dof) if theta0 is None else np.array(theta0, dtype=np.float64)
    if c is None:
        c = outlier_constant(w, len(obs), len(x_ref), feature_sigmas(feat, sigma, sigma_n))
    sig_m = float(np.mean(sigma))
    lat = build_observation_lattice(obs, obs_n, feat, residual, sigma, sigma_n)
    x_ref = np.asarray(x_ref, dtype=np.float32)
    for _ in range(iters):
        T, _, _ = forward_kinematics(tree, theta)
        x32 = np.zeros_like(x_ref)
        n32 = np.zeros_like(x_ref) if feat == 6 else None
        x64 = np.zeros((len(x_ref), 3))
        for b in range(tree.n_bodies):
            sl = slice(body_offsets[b], body_offsets[b + 1])
            mat = pose_to_mat12(T[b])
            x32[sl] = transform_f32(mat, x_ref[sl])
            if feat == 6:
                n32[sl] = transform_f32(mat, n_ref[sl], translate=False)
            R = mat.reshape(3, 4).astype(np.float64)
            x64[sl] = x_ref[sl].astype(np.float64) @ R[:, :3].T + R[:, 3]
        m0, m1, ns = estep(lat, x32, n32, feat, residual)
        A, b = normal_equations_alg1(tree, theta, x64, body_offsets, m0, m1, ns, c, sig_m, residual)
        dth = gn_step(*hold_unsupported(A, b), RIGID_PIVOT_TOL)
        theta = theta + dth
        if history is not None:
            history.append(dict(A=A, b=b, dtheta=dth, theta=theta.copy()))
    return theta
