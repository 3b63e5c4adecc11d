"""Shared helpers of the GPU parity tests: run both sides on the same seeded inputs.

Tolerances (derived from the arithmetic of the GPU path):
* lattice keys, occupancy, vertex counts: bit-exact (integer results decided by
  the same binary32 operations on both sides);
* per-vertex values: the GPU weights are binary32 differences of quantities
  bounded by 1, so each weight carries an absolute error below 4 * 2^-24;
  summed in binary64 and stored in binary32 a vertex value is within
  1e-6 * (incidences) of the binary64 oracle -> |dv| <= 1e-5 * max(1, |v0|) * L;
* E-step outputs: |dM0| <= 1e-5 * M0 + 1e-6 * max vertex mass (the second term
  bounds the weight rounding at points whose own mass is tiny); M1 and N the
  same times L = max |y| (1 for normals);
* normal equations: |dA| <= 1e-5 * sum |w J^T J| and |db| <= 1e-5 * sum |w J^T r|
  (binary32 accumulation per tile, relative to the absolute-value sums);
* poses: rotation angle <= 1e-4 rad and translation <= 1e-4 units.
"""
import math

import numpy as np

import oracle


def soa(t):
    return t.detach().cpu().numpy()


def upload(sets, normals=None):
    import paper_1811_10136_amd as fr
    return fr.Cloud.from_numpy(sets, normals)


def oracle_lattice(obs, obs_n, feat, residual, sigma, sigma_n):
    k = oracle.scale_factors(oracle.feature_sigmas(feat, sigma, sigma_n))
    return oracle.lattice_build(oracle.features(obs, obs_n, feat), oracle.splat_values(obs, obs_n, residual), k)


def assert_lattice_equal(keys, occ, vals, lat_ref, L):
    assert keys.shape == lat_ref.keys.shape, (keys.shape, lat_ref.keys.shape)
    np.testing.assert_array_equal(keys, lat_ref.keys)
    np.testing.assert_array_equal(occ, lat_ref.occ)
    ref = lat_ref.vals
    m0 = np.maximum(1.0, np.abs(ref[:, :1]))
    tol = np.concatenate([1e-5 * m0, 1e-5 * m0 * L * np.ones((1, 3)), 1e-5 * m0 * np.ones((1, ref.shape[1] - 4))],
                         axis=1)[:, : ref.shape[1]]
    err = np.abs(vals.astype(np.float64) - ref)
    bad = err > tol
    assert not bad.any(), f"{bad.sum()} lattice values out of tolerance; worst {err.max():.3e}"


def assert_estep_close(m0, m1, ns, ref_m0, ref_m1, ref_ns, vmax, L):
    tol0 = 1e-5 * np.abs(ref_m0) + 1e-6 * vmax
    e0 = np.abs(m0.astype(np.float64) - ref_m0)
    assert (e0 <= tol0).all(), f"M0: {(e0 > tol0).sum()} bad, worst {e0.max():.3e}"
    tol1 = (tol0 * L)[:, None]
    e1 = np.abs(m1.astype(np.float64) - ref_m1)
    assert (e1 <= tol1).all(), f"M1: {(e1 > tol1).sum()} bad, worst {e1.max():.3e}"
    if ref_ns is not None:
        e2 = np.abs(ns.astype(np.float64) - ref_ns)
        assert (e2 <= tol0[:, None]).all(), f"N: {(e2 > tol0[:, None]).sum()} bad, worst {e2.max():.3e}"


def abs_scales(x, m0, m1, ns, c, sigma, residual):
    """sum |w J^T J| and sum |w J^T r| of the oracle's terms (scales of the reduce tolerance)."""
    w, r, J, _ = oracle.residuals_and_jacobians(x, m0, m1, ns, c, sigma, residual)
    aJ = np.abs(J)
    A = np.einsum("i,ikp,ikq->pq", w, aJ, aJ)
    b = np.einsum("i,ikp,ik->p", w, aJ, np.abs(r))
    return A, b


def upper(A):
    iu = np.triu_indices(6)
    return A[iu]


def pose_close(T, R, tol=1e-4):
    ang = oracle.rotation_angle(T[:3, :3] @ R[:3, :3].T)
    dt = float(np.abs(T[:3, 3] - R[:3, 3]).max())
    return ang, dt, (ang <= tol and dt <= tol)
