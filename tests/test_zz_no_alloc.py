"""fr_mstep_reduce_noalloc (the reduction for callers that cannot allocate) against fr_mstep_reduce.

Same kernels and tile map on both paths, so the normal equations agree bitwise; two calls in a row, the
second smaller, check that the scratch array's leftovers from the first never leak into the second.
"""
import numpy as np
import pytest

import oracle
import synth
from _helpers import soa, upload

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1811_10136_amd as fr
    return fr


def _inputs(fr, ctx, pairs, Ts, segments=None):
    """Model cloud, transform and E-step outputs of the pairs at the poses Ts."""
    p0 = pairs[0]
    obs = upload([p.obs for p in pairs], [p.obs_n for p in pairs])
    lat = fr.Lattice(ctx, obs, fr.lattice_params(6, 7, p0.sigma, p0.sigma_n))
    model = upload([p.model for p in pairs], [p.model_n for p in pairs])
    mats = torch.from_numpy(np.concatenate([oracle.pose_to_mat12(T) for T in Ts]).astype(np.float32)).cuda()
    xf = fr.XForm(fr.FR_XF_RIGID, mats)
    M = model.n
    m0 = torch.empty(M, device="cuda")
    m1 = torch.empty(3 * M, device="cuda")
    ns = torch.empty(3 * M, device="cuda")
    fr.fr_estep(lat.h, model, xf, m0, m1, ns)
    torch.cuda.synchronize()
    lat.close()
    if segments is not None:
        # the same transforms applied per segment: each set split in two at its middle
        off = model.offsets
        seg = [0]
        rows = []
        for s in range(model.n_sets):
            mid = (int(off[s]) + int(off[s + 1])) // 2
            seg += [mid, int(off[s + 1])]
            rows += [oracle.pose_to_mat12(Ts[s])] * 2
        xf = fr.XForm(fr.FR_XF_SEGMENTED, torch.from_numpy(np.concatenate(rows).astype(np.float32)).cuda(),
                      seg_offsets=seg)
    return model, xf, m0, m1, ns


def _reduce(fn, fr, model, xf, m0, m1, ns, n_seg, c_per_set):
    jtj = torch.full((n_seg * 21,), float("nan"), dtype=torch.float64, device="cuda")
    jtr = torch.full((n_seg * 6,), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.full((n_seg * 4,), float("nan"), dtype=torch.float64, device="cuda")
    fn(model, xf, m0, m1, ns, fr.FR_PT2PL, 0.0, 0.03, jtj, jtr, st, c_per_set=c_per_set)
    torch.cuda.synchronize()
    return soa(jtj), soa(jtr), soa(st)


@pytest.mark.gpu
def test_noalloc_reduce_equals_the_allocating_one_twice(fr):
    ctx = fr.Context(0)
    big = [synth.depth_pair(s, width=320, height=240, f=262.5) for s in (11, 12, 13)]
    small = [synth.depth_pair(14, width=96, height=72, f=78.75)]
    d = np.array([0.01, -0.01, 0.005, 0.01, 0.005, -0.01])
    for pairs, segmented in [(big, True), (small, False)]:
        Ts = [p.T_gt @ oracle.se3_exp(d) for p in pairs]
        model, xf, m0, m1, ns = _inputs(fr, ctx, pairs, Ts, segments=True if segmented else None)
        n_seg = 2 * len(pairs) if segmented else len(pairs)
        c_ps = [1e-4 * (1 + s) for s in range(len(pairs))]
        print(f"[noalloc] sets={len(pairs)} M={model.n} segments={n_seg}", flush=True)
        ref = _reduce(fr.fr_mstep_reduce, fr, model, xf, m0, m1, ns, n_seg, c_ps)
        got = _reduce(fr.fr_mstep_reduce_noalloc, fr, model, xf, m0, m1, ns, n_seg, c_ps)
        for a, b in zip(ref, got):
            assert np.isfinite(a).all() and np.abs(a).max() > 0
            np.testing.assert_array_equal(a.view(np.uint64), b.view(np.uint64))
    ctx.close()


def test_noalloc_reduce_refuses_a_plan_beyond_its_scratch():
    """Host logic only: 500k empty segments need a 10 MB tile map, more than the 8 MiB scratch; the call
    fails with FR_EINVAL before it looks the scratch up or enqueues anything."""
    import ctypes
    fr = pytest.importorskip("paper_1811_10136_amd")
    n = 500_000
    off = np.zeros(n + 1, np.int64)
    dummy = np.zeros(4, np.float32)
    p = dummy.ctypes.data
    cloud = fr.fr_cloud(p, p, p, None, None, None, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n)
    prm = fr.fr_mstep_params(fr.FR_PT2PT, 0, 0.0, 0.02, None)
    out = np.zeros(8, np.float64)
    q = out.ctypes.data
    st = fr._lib.fr_mstep_reduce_noalloc(ctypes.byref(cloud), None, None, None, None, ctypes.byref(prm), q, q, q,
                                         None)
    assert st == fr.FR_EINVAL
    assert b"scratch" in fr._lib.fr_last_error()
