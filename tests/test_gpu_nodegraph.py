"""GPU parity of the node-graph path (Sec. 5.2, Eq. 21) against the oracle."""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import nodegraph as ng
from _helpers import upload

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


def _graphs(fr, p, lam):
    e = p.extra
    return (ng.Graph(e["nodes"], e["skin_idx"], e["skin_w"], e["edges"]),
            fr.NodeGraph(e["nodes"], e["skin_idx"], e["skin_w"], e["edges"], lam))


@pytest.mark.parametrize("iters", [1, 8])
def test_nodegraph_register_parity(fr, ctx, iters):
    p = synth.nodegraph_pair(6, m=20000, n_nodes=96)
    print(f"[nodegraph] M={len(p.model)} nodes=96 iters={iters}", flush=True)
    g, gg = _graphs(fr, p, 1.0)
    T = np.repeat(np.eye(4)[None], 96, 0)
    prm = fr.register_params(3, "pt2pt", p.sigma, iters=iters, w=p.w)
    st, rep = fr.fr_register_nodegraph(ctx.h, upload([p.model]), upload([p.obs]), gg, prm, T)
    ref = ng.register_nodegraph(g, p.model, None, p.obs, None, sigma=p.sigma, w=p.w, lam=1.0, iters=iters)
    assert st == 0 and rep.iterations == iters and rep.solver_residual <= 1e-10
    for k in range(96):
        ang = oracle.rotation_angle(T[k][:3, :3] @ ref[k][:3, :3].T)
        assert ang < 1e-4 and np.abs(T[k][:3, 3] - ref[k][:3, 3]).max() < 1e-4, (k, ang)


def test_nodegraph_recovers_rigid_motion(fr, ctx):
    p = synth.separated_pair(5, 500, sigma=0.01, feat=3)
    rng = np.random.default_rng(4)
    K = 12
    nodes = p.model[rng.choice(len(p.model), K, replace=False)].astype(np.float64)
    d = np.linalg.norm(p.model[:, None, :] - nodes[None], axis=-1)
    idx = np.argsort(d, 1)[:, :4]
    w = np.exp(-np.take_along_axis(d, idx, 1) ** 2 / (2 * 0.1 ** 2)) + 1e-12
    w /= w.sum(1, keepdims=True)
    ie = np.argsort(np.linalg.norm(nodes[:, None] - nodes[None], axis=-1), 1)[:, 1:5]
    edges = np.array([(j, k) for j in range(K) for k in ie[j]])
    gg = fr.NodeGraph(nodes, idx, w, edges, 1.0)
    T = np.repeat(p.extra["T0"][None], K, 0)
    prm = fr.register_params(3, "pt2pt", p.sigma, iters=12, c=0.0)
    st, _ = fr.fr_register_nodegraph(ctx.h, upload([p.model]), upload([p.obs]), gg, prm, T)
    assert st == 0
    for k in range(K):
        np.testing.assert_allclose(T[k], p.T_gt, atol=1e-5)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "nodegraph_blob100k_oracle.npz")


def _node_err(T, ref):
    ang = max(oracle.rotation_angle(T[k][:3, :3] @ ref[k][:3, :3].T) for k in range(len(T)))
    return ang, float(np.abs(T[:, :3, 3] - ref[:, :3, 3]).max())


def _T44(t34):
    T = np.repeat(np.eye(4)[None], len(t34), 0)
    T[:, :3, :4] = t34
    return T


@pytest.fixture(scope="module")
def blob():
    return synth.nodegraph_pair(0)


def test_nodegraph_full_size_20_iterations(fr, ctx, blob):
    """The node-graph workload at full size (100k points, 512 nodes), 20 EM iterations from the identity,
    against the oracle's run (stored by tests/golden/make_nodegraph_states.py)."""
    p = blob
    g, gg = _graphs(fr, p, 1.0)
    ref = np.load(GOLDEN)
    T = np.repeat(np.eye(4)[None], 512, 0)
    prm = fr.register_params(3, "pt2pt", p.sigma, iters=20, w=p.w)
    st, rep = fr.fr_register_nodegraph(ctx.h, upload([p.model]), upload([p.obs]), gg, prm, T)
    assert st == 0 and rep.iterations == 20
    ang, dt = _node_err(T, _T44(ref["T20"]))
    print(f"[error] node graph, 512 nodes, 20 iterations: node rotation {ang:.3e} rad, translation {dt:.3e} "
          f"(bounds 1e-04)", flush=True)
    assert ang < 1e-4 and dt < 1e-4, (ang, dt)


@pytest.mark.parametrize("start", [0, 10, 19])
def test_nodegraph_full_size_one_step_from_the_oracle_state(fr, ctx, blob, start):
    """One GPU iteration from the oracle's node transforms after `start` iterations equals the oracle's
    next iteration (iterations 1, 11 and 20 of the full-size run)."""
    p = blob
    g, gg = _graphs(fr, p, 1.0)
    if start == 0:
        T0 = np.repeat(np.eye(4)[None], 512, 0)
        ref = ng.register_nodegraph(g, p.model, None, p.obs, None, sigma=p.sigma, w=p.w, lam=1.0, iters=1)
    else:
        gold = np.load(GOLDEN)
        T0 = _T44(gold[f"T{start}"])
        ref = _T44(gold[f"T{start + 1}"])
    T = T0.copy()
    prm = fr.register_params(3, "pt2pt", p.sigma, iters=1, w=p.w)
    st, rep = fr.fr_register_nodegraph(ctx.h, upload([p.model]), upload([p.obs]), gg, prm, T)
    assert st == 0 and rep.solver_residual <= 1e-10
    ang, dt = _node_err(T, ref)
    assert ang < 1e-4 and dt < 1e-4, (ang, dt)


def _spread(K, seed):
    # node motions of up to 0.1 rad and 0.02 units: all different, small enough against sigma = 0.02 that
    # most moved points keep lattice support
    rng = np.random.default_rng(seed)
    return np.stack([synth.random_motion(rng, 0.1, 0.02) for _ in range(K)])


@pytest.mark.parametrize("residual", ["pt2pt", "pt2pl"])
def test_mstep_reduce_nodes_matches_the_oracle_system(fr, ctx, residual):
    """fr_mstep_reduce_nodes against the oracle's dense node system (Sec. 5.2, Eq. 21) at node transforms
    that all differ, regulariser included: every block the oracle fills is listed, values agree to the
    binary32 per-point terms' rounding, and the right-hand sides agree."""
    K = 48
    p = synth.nodegraph_pair(9, m=6000, n_nodes=K)
    e = p.extra
    lam = 0.7
    g, gg = _graphs(fr, p, lam)
    T = _spread(K, 3)
    x64, _ = ng.warp(T, g, p.model)
    x32 = x64.astype(np.float32)
    nrm = p.model_n if residual == "pt2pl" else None
    k = oracle.scale_factors(oracle.feature_sigmas(3, p.sigma, 0.5))
    obs_n = p.obs_n if residual == "pt2pl" else None
    lat = oracle.lattice_build(oracle.features(p.obs, None, 3), oracle.splat_values(p.obs, obs_n, residual), k)
    m0, m1, ns = oracle.estep(lat, x32, None, 3, residual)
    m0 = m0.astype(np.float32)
    m1 = m1.astype(np.float32)
    ns = ns.astype(np.float32) if ns is not None else None
    assert (m0 > 0).mean() > 0.5
    c, sigma = 0.05, 0.02
    A_ref, b_ref = ng.node_blocks(g, T, x32.astype(np.float64), m0.astype(np.float64), m1.astype(np.float64),
                                  None if ns is None else ns.astype(np.float64), c, sigma, residual, lam)
    dev = torch.device("cuda")
    xc = fr.Cloud.from_numpy([x32])
    t_m0 = torch.from_numpy(m0).to(dev)
    t_m1 = torch.from_numpy(np.ascontiguousarray(m1.T)).to(dev)
    t_ns = torch.from_numpy(np.ascontiguousarray(ns.T)).to(dev) if ns is not None else None
    res = fr.FR_PT2PL if residual == "pt2pl" else fr.FR_PT2PT
    kl, blocks, rhs = fr.fr_mstep_reduce_nodes(ctx.h, xc, t_m0, t_m1, t_ns, gg, T, res, c, sigma)
    B = blocks.cpu().numpy()
    A = np.zeros_like(A_ref)
    for (kk, ll), blk in zip(kl, B):
        assert kk <= ll
        A[6 * kk:6 * kk + 6, 6 * ll:6 * ll + 6] = blk
        if kk != ll:
            A[6 * ll:6 * ll + 6, 6 * kk:6 * kk + 6] = blk.T
    listed = {(int(a), int(b)) for a, b in kl}
    A4 = np.abs(A_ref).reshape(K, 6, K, 6).sum(axis=(1, 3))
    for a, b in zip(*np.nonzero(A4)):
        assert (min(a, b), max(a, b)) in listed, (a, b)
    scale = np.abs(A_ref).max()
    np.testing.assert_allclose(A, A_ref, rtol=0, atol=2e-5 * scale)
    np.testing.assert_allclose(rhs.cpu().numpy(), b_ref, rtol=0, atol=2e-5 * np.abs(b_ref).max())
    # the regulariser is part of it: without lambda the diagonal blocks differ
    assert np.abs(A_ref - ng.node_blocks(g, T, x32.astype(np.float64), m0.astype(np.float64),
                                         m1.astype(np.float64), None if ns is None else ns.astype(np.float64), c,
                                         sigma, residual, 0.0)[0]).max() > 1e-2 * scale


def test_a_node_without_support_or_edges_is_degenerate(fr, ctx):
    """With lambda = 0 a node that skins no point has an all-zero diagonal block: the GPU stops with
    FR_EDEGENERATE where the oracle's Cholesky fails."""
    p = synth.nodegraph_pair(11, m=3000, n_nodes=24)
    e = p.extra
    idx = np.array(e["skin_idx"]).copy()
    lonely = 23
    idx[idx == lonely] = 0
    w = np.array(e["skin_w"])
    g = ng.Graph(e["nodes"], idx, w, e["edges"])
    gg = fr.NodeGraph(e["nodes"], idx, w, e["edges"], 0.0)
    T = np.repeat(np.eye(4)[None], 24, 0)
    prm = fr.register_params(3, "pt2pt", p.sigma, iters=2, w=p.w)
    st, rep = fr.fr_register_nodegraph(ctx.h, upload([p.model]), upload([p.obs]), gg, prm, T)
    assert st == fr.FR_EDEGENERATE and rep.n_degenerate == 1 and rep.iterations == 1
    np.testing.assert_array_equal(T, np.repeat(np.eye(4)[None], 24, 0))     # no node moved
    with pytest.raises(oracle.Degenerate):
        ng.register_nodegraph(g, p.model, None, p.obs, None, sigma=p.sigma, w=p.w, lam=0.0, iters=2)
