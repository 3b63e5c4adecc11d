"""Pins of the oracle's lattice E-step (Sec. 4) against facts that do not come from the oracle.

* hand-worked embeddings (tests/golden/embed_hand.json),
* exact invariants of the permutohedral embedding (barycentric identity,
  remainder classes, canonical simplex shape, scaled isometry onto sum(e) = 0),
* the splat + slice result against a brute-force kernel sum that builds no
  lattice, single-point exactness, and the conservation laws of the splat.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "embed_hand.json")


def _full(keys):
    """Append the implied last coordinate (vertices lie on sum = 0)."""
    return np.concatenate([keys, -keys.sum(-1, keepdims=True)], -1).astype(np.int64)


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_hand_worked_embedding(case):
    d = len(case["p"])
    keys, b, e = oracle.embed(np.array([case["p"]], np.float32), np.ones(d, np.float32))
    np.testing.assert_allclose(e[0], np.float32(case["e"]), rtol=0, atol=1e-7)
    assert keys[0].tolist() == case["keys"]
    np.testing.assert_allclose(b[0], case["b"], rtol=0, atol=case["b_tol"])


@pytest.mark.parametrize("d", [1, 2, 3, 6, 10, 16, 32])
def test_embedding_invariants(d):
    rng = np.random.default_rng(d)
    sig = rng.uniform(0.3, 2.0, size=d)
    k = oracle.scale_factors(sig)
    f = (rng.normal(size=(20000 if d <= 16 else 5000, d)) * 4.0).astype(np.float32)
    keys, b, e = oracle.embed(f, k)
    D = d + 1
    v = _full(keys)
    # weights are a convex combination
    assert b.min() >= -1e-6
    np.testing.assert_allclose(b.sum(1), 1.0, atol=1e-12)
    # vertex k is a lattice point of remainder k
    for kk in range(D):
        assert np.all((v[:, kk] - kk) % D == 0)
    # consecutive vertices differ by a permutation of (1, ..., 1, -d): the canonical simplex
    step = v[:, 1:] - v[:, :-1]
    assert np.all((step == 1).sum(-1) == d) and np.all((step == -d).sum(-1) == 1)
    # barycentric identity: sum_k b_k v_k is the projection of e onto sum = 0
    e64 = e.astype(np.float64)
    proj = e64 - e64.mean(1, keepdims=True)
    rec = np.einsum("nk,nkj->nj", b, v.astype(np.float64))
    assert np.abs(rec - proj).max() <= 1e-12 * max(1.0, np.abs(proj).max())
    # the elevation is a scaled isometry of the normalised feature: |e|^2 = (2/3)(d+1)^2 |f/sigma|^2
    ratio = (e64 ** 2).sum(1) / ((f / sig) ** 2).sum(1)
    np.testing.assert_allclose(ratio, 2.0 / 3.0 * D * D, rtol=2e-6)
    assert np.abs(e64.sum(1)).max() <= 1e-5 * max(1.0, np.abs(e64).max())


def test_embedding_is_translation_equivariant_on_the_lattice():
    """Shifting a point by a lattice vector (in elevated space) shifts every vertex by it
    and leaves the weights unchanged.  A shift by D along feature 0 moves e by (D, -D, 0...)
    when k_0 = 1, which is a remainder-0 lattice vector."""
    rng = np.random.default_rng(7)
    for d in (2, 3, 6):
        D = d + 1
        k = np.ones(d, np.float32)
        f = rng.uniform(-3, 3, size=(2000, d)).astype(np.float32)
        f = np.round(f * 64) / 64  # exact in binary32 after the shift
        g = f.copy()
        g[:, 0] += D
        k1, b1, _ = oracle.embed(f.astype(np.float32), k)
        k2, b2, _ = oracle.embed(g.astype(np.float32), k)
        # e_0 gains D and e_1 loses D (its -1 * cf_0 term); the other coordinates are unchanged
        sh_full = np.zeros(D, np.int64)
        sh_full[0], sh_full[1] = D, -D
        np.testing.assert_array_equal(_full(k2) - _full(k1), np.broadcast_to(sh_full, _full(k1).shape))
        np.testing.assert_allclose(b1, b2, atol=1e-12)


@pytest.mark.parametrize("feat,residual", [(3, "pt2pt"), (3, "pt2pl"), (6, "pt2pl"), (6, "pt2pt")])
def test_splat_slice_equals_brute_force(feat, residual):
    p = synth.random_cloud_pair(11 + feat, 180, 240, feat=feat, residual=residual)
    k = oracle.scale_factors(oracle.feature_sigmas(feat, p.sigma, p.sigma_n))
    fy = oracle.features(p.obs, p.obs_n, feat)
    vals = oracle.splat_values(p.obs, p.obs_n, residual)
    lat = oracle.lattice_build(fy, vals, k)
    fx = oracle.features(p.model, p.model_n, feat)
    got = oracle.lattice_slice(lat, fx)
    ref = oracle.brute_force_lattice_sum(fy, vals, fx, k)
    assert (ref[:, 0] > 0).mean() > 0.3
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))


def test_splat_conservation_and_sorting():
    p = synth.random_cloud_pair(3, 10, 500, feat=6, residual="pt2pl")
    k = oracle.scale_factors(oracle.feature_sigmas(6, p.sigma, p.sigma_n))
    lat = oracle.lattice_build(oracle.features(p.obs, p.obs_n, 6), oracle.splat_values(p.obs, p.obs_n, "pt2pl"), k)
    assert lat.occ.sum() == 7 * 500
    np.testing.assert_allclose(lat.vals[:, 0].sum(), 500.0, rtol=1e-12)
    # each vertex value equals sum of b * v over its incidences: total position mass = sum of y
    np.testing.assert_allclose(lat.vals[:, 1:4].sum(0), p.obs.astype(np.float64).sum(0), rtol=1e-10, atol=1e-10)
    keys = [tuple(r) for r in lat.keys]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    assert lat.vals[:, 0].min() >= 0


@pytest.mark.parametrize("feat", [3, 6])
def test_single_observation_point_is_exact(feat):
    rng = np.random.default_rng(feat)
    y = rng.uniform(-0.2, 0.2, size=(1, 3)).astype(np.float32)
    ny = rng.normal(size=(1, 3))
    ny = (ny / np.linalg.norm(ny)).astype(np.float32)
    sigma = (0.05, 0.05, 0.05)
    k = oracle.scale_factors(oracle.feature_sigmas(feat, sigma, 0.5))
    lat = oracle.lattice_build(oracle.features(y, ny, feat), oracle.splat_values(y, ny, "pt2pl"), k)
    assert lat.n_vertices == feat + 1
    x = (y + rng.normal(scale=0.02, size=(400, 3))).astype(np.float32)
    nx = np.repeat(ny, 400, 0)
    g = oracle.lattice_slice(lat, oracle.features(x, nx, feat))
    sup = g[:, 0] > 0
    assert sup.sum() > 50
    np.testing.assert_allclose(g[sup, 1:4] / g[sup, :1], np.broadcast_to(y.astype(np.float64), (sup.sum(), 3)), atol=1e-12)
    np.testing.assert_allclose(g[sup, 4:7] / g[sup, :1], np.broadcast_to(ny.astype(np.float64), (sup.sum(), 3)), atol=1e-12)
    # the kernel at the point itself is sum_k b_k^2, between 1/(d+1) and 1
    g0 = oracle.lattice_slice(lat, oracle.features(y, ny, feat))
    assert 1.0 / (feat + 1) - 1e-12 <= g0[0, 0] <= 1.0 + 1e-12


@pytest.mark.parametrize("d,bound,spread", [(3, 2.45, 1.5), (6, 3.21, 0.8)])
def test_kernel_support_is_bounded(d, bound, spread):
    """Two points share a lattice vertex only if they are within two simplex edges;
    with the sqrt(2/3)(d+1) scale the longest edge is sqrt(1.5 k (d+1-k)/(d+1)) sigma."""
    longest = max(math.sqrt(1.5 * kk * (d + 1 - kk) / (d + 1)) for kk in range(1, d + 1))
    assert abs(2 * longest - bound) < 0.01
    rng = np.random.default_rng(d)
    k = np.asarray(oracle.scale_factors(np.ones(d)))
    y = rng.uniform(-2, 2, size=(300, d)).astype(np.float32)
    x = (y + rng.normal(size=(300, d)) * spread).astype(np.float32)
    K = oracle.brute_force_lattice_sum(y, np.eye(300), x, k)   # K[i, j] = K(x_i, y_j)
    dist = np.linalg.norm(x[:, None, :].astype(np.float64) - y[None, :, :], axis=-1)
    assert np.all(K[dist > bound] == 0.0)
    assert (K > 0).sum() > 100


def test_touched_vertices_and_empty_inputs():
    p = synth.random_cloud_pair(5, 300, 300)
    k = oracle.scale_factors(oracle.feature_sigmas(3, p.sigma, p.sigma_n))
    lat = oracle.lattice_build(oracle.features(p.obs, None, 3), oracle.splat_values(p.obs, None, "pt2pt"), k)
    out, nt = oracle.lattice_slice(lat, oracle.features(p.model, None, 3), return_touched=True)
    assert 0 < nt <= lat.n_vertices
    empty = oracle.lattice_build(np.zeros((0, 3), np.float32), np.zeros((0, 4)), k)
    assert empty.n_vertices == 0
    g = oracle.lattice_slice(empty, oracle.features(p.model, None, 3))
    assert np.all(g == 0)
    assert oracle.lattice_slice(lat, np.zeros((0, 3), np.float32)).shape == (0, 4)


def test_pinned_transform_is_binary32_in_order():
    rng = np.random.default_rng(0)
    T = synth.random_motion(rng, 0.5, 0.3)
    mat = oracle.pose_to_mat12(T)
    p = rng.normal(size=(1000, 3)).astype(np.float32)
    got = oracle.transform_f32(mat, p)
    R = mat.reshape(3, 4)
    ref = ((R[:, 0] * p[:, :1] + R[:, 1] * p[:, 1:2]) + R[:, 2] * p[:, 2:3]) + R[:, 3]   # numpy binary32 ops
    np.testing.assert_array_equal(got, ref.astype(np.float32))
    np.testing.assert_allclose(got, p @ T[:3, :3].T + T[:3, 3], atol=1e-5)
