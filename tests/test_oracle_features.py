"""Pins of the oracle's descriptor E-step (Sec. 3.3 "Features", Eq. 8) and registration by descriptors.

The lattice code is the same at every dimension; these tests pin it at descriptor dimensions (the
embedding invariants at d = 16 and 32 live in test_oracle_lattice.py): splat + slice against the
brute-force kernel sum at d = 8, 16 and 32, the outlier constant against the position case, and
recovery of arbitrary rotations from descriptors alone.  (A Monte Carlo check of the kernel's moment,
as at d = 3 and 6, does not converge at d = 16: the compact kernel leaves an effective sample size of
a few dozen in 8000 draws.)
"""
import math

import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("dim", [8, 16, 32])
def test_descriptor_splat_slice_equals_brute_force(dim):
    p = synth.feature_pair(5, m=400, dim=dim, clutter=0.2)
    e = p.extra
    lat = oracle.feature_lattice(p.obs, e["obs_feat"], e["sigma_f"])
    got = oracle.lattice_slice(lat, e["model_feat"])
    k = oracle.scale_factors(np.full(dim, e["sigma_f"]))
    ref = oracle.brute_force_lattice_sum(e["obs_feat"], oracle.splat_values(p.obs, None, "pt2pt"), e["model_feat"], k)
    assert (ref[:, 0] > 0).mean() > 0.4
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("seed", [3, 4])
def test_descriptors_recover_large_rotations(seed):
    p = synth.feature_pair(seed, m=6000, dim=16)
    e = p.extra
    ang = math.degrees(oracle.rotation_angle(p.T_gt[:3, :3]))
    assert ang > 100                                        # far outside any local basin
    T = oracle.register_rigid_features(p.model, e["model_feat"], p.obs, e["obs_feat"], sigma_f=e["sigma_f"], w=p.w,
                                       iters=20)
    assert oracle.alignment_error(T, p.T_gt, p.model) < 1e-3
