"""GPU parity of the articulated path (Sec. 5.1, Alg. 1) against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from oracle import articulated as art
from _helpers import soa, upload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1811_10136_amd as fr
    return fr


@pytest.fixture(scope="module")
def ctx(fr):
    c = fr.Context(0)
    yield c
    c.close()


def _trees(fr, p):
    t = p.extra["tree"]
    return art.Tree(t.parent, t.dof_offset, t.origin, t.axis), fr.KinematicTree(t.parent, t.dof_offset, t.origin,
                                                                                    t.axis)


def test_forward_kinematics_and_step_match_oracle(fr, ctx):
    p = synth.articulated_pair(5, m=2000)
    tree, ktree = _trees(fr, p)
    B, n = tree.n_bodies, tree.n_dof
    th0 = p.extra["theta0"]
    theta = torch.tensor(th0, dtype=torch.float64, device="cuda")
    mats = torch.zeros(B * 12, dtype=torch.float32, device="cuda")
    fr.fr_articulated_step(ctx.h, ktree, None, None, theta, mats)
    T, _, _ = art.forward_kinematics(tree, th0)
    ref = np.stack([T[b, :3, :4] for b in range(B)]).reshape(-1)
    np.testing.assert_allclose(soa(mats), ref, atol=2e-7)
    np.testing.assert_array_equal(soa(theta), th0)
    # one Gauss-Newton step from random per-body sums
    rng = np.random.default_rng(1)
    S, g = [], []
    for b in range(B):
        G = rng.normal(size=(6, 6))
        S.append(G @ G.T + 0.5 * np.eye(6))
        g.append(rng.normal(size=6))
    iu = np.triu_indices(6)
    jtj = torch.tensor(np.concatenate([Sb[iu] for Sb in S]), dtype=torch.float64, device="cuda")
    jtr = torch.tensor(np.concatenate(g), dtype=torch.float64, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    fr.fr_articulated_step(ctx.h, ktree, jtj, jtr, theta, mats, status)
    Jsp = art.spatial_jacobians(tree, th0)
    A = sum(Jsp[b].T @ S[b] @ Jsp[b] for b in range(B))
    bb = sum(Jsp[b].T @ g[b] for b in range(B))
    th1 = th0 + oracle.gn_step(A, bb)
    assert int(soa(status)[0]) == 0
    np.testing.assert_allclose(soa(theta), th1, rtol=0, atol=1e-9 * max(1.0, np.abs(th1 - th0).max()))
    T1, _, _ = art.forward_kinematics(tree, th1)
    np.testing.assert_allclose(soa(mats), np.stack([T1[b, :3, :4] for b in range(B)]).reshape(-1), atol=2e-7)


def test_articulated_register_parity(fr, ctx):
    # 60k points, 20 bodies, 32 DOF, 15 iterations; a seed whose registration settles (from some
    # starts the occluded tree drifts, and a drifting run is no test of agreement)
    p = synth.articulated_pair(1)
    print(f"[articulated] M={len(p.model)} N={len(p.obs)}", flush=True)
    tree, ktree = _trees(fr, p)
    bo = p.extra["body_offsets"]
    th = p.extra["theta0"].copy()
    prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=p.iters, w=p.w)
    st, rep = fr.fr_register_articulated(ctx.h, upload([p.model], [p.model_n]), bo, upload([p.obs], [p.obs_n]),
                                         ktree, prm, th)
    ref = art.register_articulated(tree, p.model, p.model_n, bo, p.obs, p.obs_n, feat=6, residual="pt2pl",
                                   sigma=p.sigma, sigma_n=p.sigma_n, w=p.w, iters=p.iters, theta0=p.extra["theta0"])
    assert st == 0 and rep.iterations == p.iters
    print(f"[error] articulated, 32 DOF, {p.iters} iterations: joint angles, max |d theta| (rad): "
          f"{np.abs(th - ref).max():.3e} (bound 1e-04)", flush=True)
    assert np.abs(th - ref).max() < 1e-4, np.abs(th - ref).max()
    # and it is a registration: the error to the ground truth shrinks
    assert np.abs(th - p.extra["theta_gt"]).mean() < np.abs(p.extra["theta0"] - p.extra["theta_gt"]).mean()


def test_articulated_exact_recovery(fr, ctx):
    from test_oracle_articulated import separated_articulated
    p, tree = separated_articulated(4)
    t = p.extra["tree"]
    ktree = fr.KinematicTree(t.parent, t.dof_offset, t.origin, t.axis)
    th = p.extra["theta0"].copy()
    prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=10, c=0.0)
    st, _ = fr.fr_register_articulated(ctx.h, upload([p.model], [p.model_n]), p.extra["body_offsets"],
                                       upload([p.obs], [p.obs_n]), ktree, prm, th)
    assert st == 0
    assert np.abs(th - p.extra["theta_gt"]).max() < 1e-5


def test_articulated_holds_dofs_without_support(fr, ctx):
    """The last (leaf) body has no model points: its DOFs stay put on the device as in the oracle."""
    from test_oracle_articulated import separated_articulated
    p, tree = separated_articulated(4)
    t = p.extra["tree"]
    ktree = fr.KinematicTree(t.parent, t.dof_offset, t.origin, t.axis)
    bo = p.extra["body_offsets"]
    B = tree.n_bodies
    n_keep = int(bo[B - 1])
    bo_full = np.concatenate([bo[:B], [bo[B - 1]]])
    th0 = p.extra["theta0"]
    th = th0.copy()
    prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=5, c=0.0)
    st, _ = fr.fr_register_articulated(ctx.h, upload([p.model[:n_keep]], [p.model_n[:n_keep]]), bo_full,
                                       upload([p.obs], [p.obs_n]), ktree, prm, th)
    ref = art.register_articulated(tree, p.model[:n_keep], p.model_n[:n_keep], bo_full, p.obs, p.obs_n, feat=6,
                                   residual="pt2pl", sigma=p.sigma, sigma_n=p.sigma_n, c=0.0, iters=5, theta0=th0)
    nd = int(tree.dof_offset[B - 1])
    assert st == 0
    np.testing.assert_array_equal(th[nd:], th0[nd:])
    assert np.abs(th - ref).max() < 1e-4, np.abs(th - ref).max()


@pytest.mark.parametrize("seed", [0, 2, 3, 4])
def test_articulated_one_step_from_oracle_states(fr, ctx, seed):
    """Trees of four more seeds (60k points, 20 bodies, 32 DOF): one GPU iteration from the oracle's joint
    angles before iterations 0, 4, 9 and 14 lands on the oracle's next angles (1e-4 rad).  Seeds 0 and 4
    drift away from the ground truth under occlusion -- on both sides, so the single steps still compare --
    and seeds 2 and 3 settle, where the whole 15-iteration GPU run also follows the oracle's (1e-3 rad)."""
    p = synth.articulated_pair(seed)
    print(f"[articulated-seed] seed={seed} M={len(p.model)} N={len(p.obs)}", flush=True)
    tree, ktree = _trees(fr, p)
    bo = p.extra["body_offsets"]
    hist = []
    ref = art.register_articulated(tree, p.model, p.model_n, bo, p.obs, p.obs_n, feat=6, residual="pt2pl",
                                   sigma=p.sigma, sigma_n=p.sigma_n, w=p.w, iters=p.iters, theta0=p.extra["theta0"],
                                   history=hist)
    model, obs = upload([p.model], [p.model_n]), upload([p.obs], [p.obs_n])
    one = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=1, w=p.w)
    for k in (0, 4, 9, 14):
        th = (p.extra["theta0"] if k == 0 else hist[k - 1]["theta"]).copy()
        st, rep = fr.fr_register_articulated(ctx.h, model, bo, obs, ktree, one, th)
        assert st == 0 and rep.iterations == 1
        err = np.abs(th - hist[k]["theta"]).max()
        assert err < 1e-4, (k, err)
    if seed in (2, 3):
        th = p.extra["theta0"].copy()
        prm = fr.register_params(6, "pt2pl", p.sigma, p.sigma_n, iters=p.iters, w=p.w)
        st, rep = fr.fr_register_articulated(ctx.h, model, bo, obs, ktree, prm, th)
        assert st == 0 and rep.iterations == p.iters
        assert np.abs(th - ref).max() < 1e-3, np.abs(th - ref).max()
