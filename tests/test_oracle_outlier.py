"""Pins of the outlier constant c of Eq. (7) in the units of the lattice sums (Sec. 3.1, Eq. 4-7).

Eq. (4) mixes the N Gaussian PDFs of the observation (unit mass each) with a uniform component, and
Eq. (7)'s weight M0 / (M0 + c) compares their sum with c = w/(1-w) N/M.  The lattice sums a kernel
K(x, y) = sum_v b_v(x) b_v(y) whose mass is not one, so the oracle scales c by that mass
(oracle.kernel_mass).  These tests pin the mass against numerical integration of the brute-force
kernel (no lattice built), and the resulting weights against brute-force posteriors of normalised
Gaussian PDFs on a cloud of uniform density, where both reduce to rho / (rho + c).
"""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("d,sig", [(2, [0.03, 0.05]), (3, [0.02, 0.02, 0.02]), (3, [0.01, 0.03, 0.02]),
                                   (6, [0.02, 0.02, 0.02, 0.5, 0.5, 0.5])])
def test_kernel_mass_equals_its_integral(d, sig):
    # importance sampling of x ~ N(y, (0.6 sigma)^2) (the kernel's own spread is sigma / 2 per axis and its
    # support is compact, so the weights K / q stay bounded)
    rng = np.random.default_rng(d)
    sig = np.asarray(sig)
    k = oracle.scale_factors(sig)
    est = []
    for t in range(4):
        y = (rng.uniform(-1, 1, (1, d)) * sig * 3).astype(np.float32)
        s = 0.6 * sig
        x = y.astype(np.float64) + rng.normal(size=(200_000, d)) * s
        q = np.exp(-0.5 * np.sum(((x - y) / s) ** 2, axis=1)) / ((2 * math.pi) ** (d / 2) * np.prod(s))
        K = oracle.brute_force_lattice_sum(y, np.ones((1, 1)), x.astype(np.float32), k)[:, 0]
        est.append(np.mean(K / q))
    H = oracle.kernel_mass(sig)
    assert abs(np.mean(est) / H - 1.0) < 0.01, (np.mean(est), H)
    # the normaliser of a Gaussian of the paper's sigma, (2 pi)^(d/2) prod sigma, is not the mass
    assert (2 * math.pi) ** (d / 2) * np.prod(sig) > 5 * H


def _uniform_cloud(rng, n, lo, hi):
    return rng.uniform(lo, hi, (n, len(lo))).astype(np.float32)


def test_weight_matches_normalised_gaussian_posterior_on_uniform_density():
    # Observation: N points of uniform density rho in a box; query points well inside it (beyond the
    # kernel's support and 8 Gaussian std from the faces).  There, M0 / mass and the sum of normalised
    # Gaussian PDFs both estimate rho, so the lattice weight M0 / (M0 + c) and the Gaussian posterior
    # sum N / (sum N + c_pdf) agree, for every outlier ratio w.
    rng = np.random.default_rng(7)
    sig = np.array([0.02, 0.02, 0.02])
    L, N, M = 0.4, 60_000, 60_000
    y = _uniform_cloud(rng, N, [0, 0, 0], [L, L, L])
    rho = N / L ** 3
    q = _uniform_cloud(rng, 1500, [0.1, 0.1, 0.1], [L - 0.1, L - 0.1, L - 0.1])
    k = oracle.scale_factors(sig)
    lat = oracle.lattice_build(y, np.ones((N, 1)), k)
    m0 = oracle.lattice_slice(lat, q)[:, 0]
    assert abs(m0.mean() / (rho * oracle.kernel_mass(sig)) - 1.0) < 0.03
    # normalised Gaussian PDFs of the kernel's own per-axis variance sigma^2 / 4
    s = sig / 2
    g = np.zeros(len(q))
    for i in range(0, N, 10_000):
        dd = (q[:, None, :].astype(np.float64) - y[None, i:i + 10_000, :]) / s
        g += np.exp(-0.5 * np.sum(dd * dd, axis=2)).sum(axis=1)
    g /= (2 * math.pi) ** 1.5 * np.prod(s)
    assert abs(g.mean() / rho - 1.0) < 0.03
    for target in (0.2, 0.5, 0.8):
        # w such that the paper's c = w/(1-w) N/M puts the uniform-density posterior at `target`
        c_pdf = rho * (1 - target) / target
        w = c_pdf / (1 + c_pdf)
        assert math.isclose(w / (1 - w) * N / M, c_pdf, rel_tol=1e-9)
        c = oracle.outlier_constant(w, N, M, sig)
        post_lat = np.mean(m0 / (m0 + c))
        post_gauss = np.mean(g / (g + c_pdf))
        assert abs(post_lat - target) < 0.04, (target, post_lat)
        assert abs(post_lat - post_gauss) < 0.04, (target, post_lat, post_gauss)
        # the Gaussian normaliser in place of the mass moves the weight far off
        c_bad = w / (1 - w) * N / M * (2 * math.pi) ** 1.5 * np.prod(sig)
        assert abs(np.mean(m0 / (m0 + c_bad)) - target) > 0.15


def test_blurred_kernel_mass_on_uniform_density():
    # The uncustomised filter (splat of [Y, X], blur, scale 1 / (1 + 2^-d), slice) keeps the splatted
    # mass inside a dense cloud: M0 averages rho times kernel_mass(..., blurred=True).
    rng = np.random.default_rng(11)
    sig = np.array([0.03, 0.03, 0.03])
    L, N = 0.45, 40_000
    y = _uniform_cloud(rng, N, [0, 0, 0], [L, L, L])
    q = _uniform_cloud(rng, 800, [0.15, 0.15, 0.15], [L - 0.15, L - 0.15, L - 0.15])
    m0, _, _ = oracle.estep_blurred(y, None, q, None, 3, "pt2pt", oracle.scale_factors(sig))
    rho = N / L ** 3
    assert abs(m0.mean() / (rho * oracle.kernel_mass(sig, blurred=True)) - 1.0) < 0.03
    assert math.isclose(oracle.kernel_mass(sig, blurred=True), oracle.kernel_mass(sig) / (1 + 2.0 ** -3),
                        rel_tol=1e-14)


def test_feature_outlier_constant_is_the_same_rule():
    c3 = oracle.feature_outlier_constant(0.2, 900, 1000, 0.03, 3)
    assert c3 == pytest.approx(oracle.outlier_constant(0.2, 900, 1000, [0.03, 0.03, 0.03]), rel=1e-14)
    assert oracle.feature_outlier_constant(0.0, 900, 1000, 0.05, 16) == 0.0
    assert oracle.feature_outlier_constant(0.5, 10, 10, 0.05, 16) == pytest.approx(
        oracle.kernel_mass(np.full(16, 0.05)), rel=1e-14)
