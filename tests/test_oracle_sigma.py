"""Pins of the oracle's optimised variance (Sec. 3.3, sigma as a decision variable; Tab. 1 "updated sigma").

The closed form is that of the Coherent Point Drift M-step.  It is pinned against
the double sum over point pairs that defines it, against a numerical minimiser of
the EM objective it solves, against the single-pair closed form, and the kernel
moment that links the lattice scale to the Gaussian's variance is measured by
Monte Carlo on the brute-force kernel (no lattice built).
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle
import synth


def _kernel(y, x, k):
    """K(x, y) for one pair by the brute-force shared-vertex sum."""
    return oracle.brute_force_lattice_sum(y[None], np.ones((1, 1)), x[None], k)[0, 0]


@pytest.mark.parametrize("d", [3, 6])
def test_lattice_kernel_axis_variance_is_a_quarter_of_the_scale_squared(d):
    """Importance-sampled second moment of K(y + r, y) over offsets r, y spread over many cells:
    per axis it is s^2 / 4, the moment the update divides by."""
    rng = np.random.default_rng(7 + d)
    s = np.array([0.8, 1.0, 1.3, 0.9, 1.1, 0.7][:d])
    k = oracle.scale_factors(s)
    n = 6000 if d == 3 else 9000
    tau = 0.55 * s
    num = np.zeros(d)
    den = 0.0
    for _ in range(n):
        y = rng.uniform(-40.0, 40.0, size=d).astype(np.float32)
        r = rng.normal(size=d) * tau
        x = (y.astype(np.float64) + r).astype(np.float32)
        r32 = x.astype(np.float64) - y.astype(np.float64)
        q = math.exp(-0.5 * float(np.sum((r32 / tau) ** 2)))   # proposal density up to a constant
        kv = _kernel(y, x, k) / q
        num += kv * r32 ** 2
        den += kv
    var = num / den / s ** 2
    assert np.all(np.abs(var - oracle.LATTICE_KERNEL_AXIS_VAR) < 0.03), var
    assert abs(var.mean() - oracle.LATTICE_KERNEL_AXIS_VAR) < 0.012, var


def test_m2_channel_matches_brute_force():
    rng = np.random.default_rng(3)
    y = rng.uniform(-0.2, 0.2, size=(300, 3)).astype(np.float32)
    x = (y[:120] + rng.normal(scale=0.01, size=(120, 3))).astype(np.float32)
    k = oracle.scale_factors([0.03, 0.03, 0.03])
    vals = oracle.splat_values(y, None, "pt2pt", m2=True)
    assert vals.shape == (300, 5)
    lat = oracle.lattice_build(y, vals, k)
    m0, m1, ns, m2 = oracle.estep(lat, x, None, 3, "pt2pt", m2=True)
    assert ns is None
    yy = np.sum(y.astype(np.float64) ** 2, axis=1, keepdims=True)
    bf = oracle.brute_force_lattice_sum(y, yy, x, k)[:, 0]
    np.testing.assert_allclose(m2, bf, rtol=1e-12, atol=1e-15)
    assert (m0 > 0).mean() > 0.9


def _gaussian_moments(x, y, var):
    N = np.exp(-0.5 * np.sum((x[:, None, :] - y[None, :, :]) ** 2, axis=2) / var)
    return N, N.sum(1), N @ y, N @ np.sum(y * y, axis=1)


def test_variance_terms_match_the_cpd_double_sum():
    rng = np.random.default_rng(11)
    x = rng.normal(size=(40, 3))
    y = rng.normal(size=(55, 3)) + 0.3
    N, m0, m1, m2 = _gaussian_moments(x, y, 0.5)
    c = 0.07
    P = N / (N.sum(1, keepdims=True) + c)
    d2 = np.sum((x[:, None, :] - y[None, :, :]) ** 2, axis=2)
    first, second = oracle.variance_terms(x, m0, m1, m2, c)
    assert first == pytest.approx(float(np.sum(P * d2)), rel=1e-12)
    assert second == pytest.approx(float(np.sum(P)), rel=1e-12)
    # points without support are left out
    m0z = m0.copy()
    m0z[:5] = 0.0
    f2, s2 = oracle.variance_terms(x, m0z, m1, m2, c)
    assert s2 == pytest.approx(float(np.sum(P[5:])), rel=1e-12)
    assert f2 == pytest.approx(float(np.sum(P[5:] * d2[5:])), rel=1e-12)


def test_closed_form_minimises_the_em_objective():
    """With the posterior held, the sigma part of the expected negative log-likelihood,
    sum_ik P_ik |x_i - y_k|^2 / (2 v) + 3/2 sum_ik P_ik log v, is minimised at v = first / (3 second)."""
    rng = np.random.default_rng(12)
    x = rng.normal(size=(30, 3)) * 0.4
    y = rng.normal(size=(35, 3)) * 0.4
    N, m0, m1, m2 = _gaussian_moments(x, y, 0.2)
    c = 0.02
    P = N / (N.sum(1, keepdims=True) + c)
    d2 = np.sum((x[:, None, :] - y[None, :, :]) ** 2, axis=2)

    def q(v):
        return float(np.sum(P * d2)) / (2.0 * v) + 1.5 * float(np.sum(P)) * math.log(v)

    best = minimize_scalar(q, bounds=(1e-4, 10.0), method="bounded", options={"xatol": 1e-10}).x
    first, second = oracle.variance_terms(x, m0, m1, m2, c)
    assert first / (3.0 * second) == pytest.approx(best, rel=1e-5)


def test_one_observation_gives_the_squared_distance_over_three():
    y = np.array([[0.011, -0.004, 0.02]], np.float32)
    x = np.array([[0.016, -0.001, 0.017]], np.float32)
    k = oracle.scale_factors([0.02, 0.02, 0.02])
    lat = oracle.lattice_build(y, oracle.splat_values(y, None, "pt2pt", m2=True), k)
    m0, m1, _, m2 = oracle.estep(lat, x, None, 3, "pt2pt", m2=True)
    assert m0[0] > 0
    first, second = oracle.variance_terms(x.astype(np.float64), m0, m1, m2, 0.0)
    d2 = float(np.sum((x.astype(np.float64) - y.astype(np.float64)) ** 2))
    assert second == pytest.approx(1.0, rel=1e-12)
    assert first / (3 * second) == pytest.approx(d2 / 3.0, rel=1e-6)


def test_updated_sigma_recovers_the_pose_and_tracks_the_noise():
    """A start 8 cm off: the fixed-sigma loop at the start scale stalls, the updated scale first
    widens (the misalignment), then shrinks to the noise level (Tab. 1: updated sigma needs fewer
    iterations)."""
    noise = 0.01
    p = synth.ellipsoid_pair(2, m=2000, max_angle_deg=10, max_trans=0.05, noise=noise)
    hist = []
    T, s = oracle.register_rigid_sigma(p.model, p.model_n, p.obs, p.obs_n, feat=3, residual="pt2pt", sigma0=0.02,
                                       sigma_min=1e-3, w=p.w, iters=25, T0=np.eye(4), history=hist)
    err = [oracle.alignment_error(h["T"], p.T_gt, p.model) for h in hist]
    assert err[0] > 0.05 and err[-1] < 2e-3
    sig = [h["sigma"] for h in hist]
    assert max(sig) > 0.04                        # widened while misaligned
    assert 0.6 * noise < s / 2.0 < 1.2 * noise    # the Gaussian's std (s / 2) against the noise
    Tf = oracle.register_rigid(p.model, p.model_n, p.obs, p.obs_n, feat=3, residual="pt2pt", sigma=p.sigma, w=p.w,
                               iters=25, T0=np.eye(4))
    assert oracle.alignment_error(Tf, p.T_gt, p.model) > 10 * err[-1]


def test_noise_free_pair_drives_sigma_to_the_floor():
    p = synth.separated_pair(5, 300)
    hist = []
    T, s = oracle.register_rigid_sigma(p.model, p.model_n, p.obs, p.obs_n, feat=3, residual="pt2pt", sigma0=0.02,
                                       sigma_min=0.004, w=0.0, iters=12, T0=p.extra["T0"], history=hist)
    assert s == 0.004
    assert np.abs(T - p.T_gt).max() < 1e-6
    assert all(b["sigma"] <= a["sigma"] + 1e-12 for a, b in zip(hist, hist[1:]))
