"""Pins of the oracle's uncustomised filter: splat of [Y, X], blur along the d+1 lattice directions,
slice at X (the cited Adams et al. permutohedral filter; Sec. 4.2 customises it, Sec. 3.1 notes that it
must be rebuilt every iteration because X moves).

The blur is pinned by its impulse response, enumerated independently as a sum over the 3^(d+1) paths of
the separable [1/4, 1/2, 1/4] stencil; the whole filter by its kernel's second moment, s^2 per axis for a
lattice of scale s (splat and slice give s^2/4, the d+1 blur passes add 3 s^2/4), by Monte Carlo; and the
EM loop built on it by recovery of a known motion.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth


def _directions(d):
    """The d+1 lattice directions as full (d+1)-vectors: +1 everywhere, -d at coordinate j."""
    E = np.ones((d + 1, d + 1), dtype=np.int64)
    for j in range(d + 1):
        E[j, j] = -d
    return E


@pytest.mark.parametrize("d", [2, 3, 6])
def test_blur_impulse_response_matches_the_enumerated_stencil(d):
    E = _directions(d)
    weight = {-1: 0.25, 0: 0.5, 1: 0.25}
    expected = {}
    for a in itertools.product((-1, 0, 1), repeat=d + 1):
        pos = tuple(int(v) for v in np.asarray(a) @ E)
        expected[pos] = expected.get(pos, 0.0) + math.prod(weight[x] for x in a)
    # the lattice: every position the stencil reaches, keyed by its first d coordinates
    keys = np.array([p[:d] for p in expected], dtype=np.int32)     # centred on the origin
    order = np.lexsort(keys.T[::-1])
    keys = np.ascontiguousarray(keys[order])
    vals = np.zeros((len(keys), 1))
    origin = np.where((keys == 0).all(axis=1))[0][0]
    vals[origin, 0] = 1.0
    lat = oracle.Lattice(keys, np.ones(len(keys), np.int32), vals, np.ones(d, np.float32), d)
    out = oracle.lattice_blur(lat)
    alpha = 1.0 / (1.0 + 2.0 ** (-d))
    got = {tuple(int(v) for v in k): out.vals[i, 0] for i, k in enumerate(keys)}
    for p, e in expected.items():
        assert got[p[:d]] == pytest.approx(alpha * e, rel=1e-12, abs=1e-15), p
    assert sum(got.values()) == pytest.approx(alpha, rel=1e-12)    # mass kept: every neighbour exists


def test_blurred_kernel_has_the_lattice_scale_as_its_standard_deviation():
    """One valued observation among dense zero-valued queries (so every vertex of the support exists):
    the second moment of K(x, y) over x is s^2 per axis."""
    rng = np.random.default_rng(3)
    s = np.array([0.9, 1.0, 1.2])
    k = oracle.scale_factors(s)
    R = 4.2 * s
    mom = []
    for _ in range(24):
        y = rng.uniform(-30, 30, size=(1, 3)).astype(np.float32)
        r = rng.uniform(-1.0, 1.0, size=(40000, 3)) * R
        x = (y.astype(np.float64) + r).astype(np.float32)
        lat = oracle.lattice_blur(oracle.joint_lattice(y, np.ones((1, 1)), x, k))
        K = oracle.lattice_slice(lat, x)[:, 0]
        r32 = x.astype(np.float64) - y.astype(np.float64)
        assert K[np.abs(r32 / s).max(axis=1) > 4.0].max() < 1e-3 * K.max()   # support inside the cube
        mom.append((K[:, None] * r32 ** 2).sum(0) / K.sum() / s ** 2)
    mom = np.mean(mom, axis=0)
    assert np.all(np.abs(mom - 1.0) < 0.04) and abs(mom.mean() - 1.0) < 0.02, mom   # standard error ~0.01


def test_blurred_filter_tracks_the_gaussian_weighted_mean():
    """On a dense cloud the filter's M1 / M0 follows the exact Gaussian-weighted mean of the observations
    (the quantity the E-step of Eq. 6 asks for) to a small fraction of sigma."""
    p = synth.random_cloud_pair(9, 600, 4000, extent=0.15, sigma=0.02, feat=3, residual="pt2pt")
    k = oracle.scale_factors([0.02, 0.02, 0.02])
    m0, m1, _ = oracle.estep_blurred(p.obs, None, p.model, None, 3, "pt2pt", k)
    y = p.obs.astype(np.float64)
    x = p.model.astype(np.float64)
    G = np.exp(-0.5 * np.sum((x[:, None, :] - y[None, :, :]) ** 2, axis=2) / 0.02 ** 2)
    exact = G @ y / G.sum(1, keepdims=True)
    sup = G.sum(1) > 1.0
    err = np.linalg.norm(m1[sup] / m0[sup, None] - exact[sup], axis=1)
    # measured 0.034 sigma (median) and 0.08 sigma (95th percentile); the filter without blur is off by
    # 0.19 sigma (median) at scale sigma and 0.20 sigma at scale 2 sigma
    assert np.median(err) < 0.06 * 0.02 and np.percentile(err, 95) < 0.15 * 0.02, (np.median(err), err.max())


def test_blurred_em_recovers_a_motion():
    p = synth.ellipsoid_pair(4, m=2000, max_angle_deg=6, max_trans=0.03)
    T = oracle.register_rigid_blurred(p.model, p.model_n, p.obs, p.obs_n, feat=3, residual="pt2pt", sigma=p.sigma,
                                      w=p.w, iters=30, T0=np.eye(4))
    assert oracle.alignment_error(np.eye(4), p.T_gt, p.model) > 0.03
    assert oracle.alignment_error(T, p.T_gt, p.model) < 2e-3
