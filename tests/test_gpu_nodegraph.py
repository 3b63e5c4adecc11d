"""GPU parity of the node-graph path (Sec. 5.2, Eq. 21) against the oracle."""
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


def test_nodegraph_full_size_runs(fr, ctx):
    """The node-graph workload at full size (100k points, 512 nodes): two iterations against the oracle."""
    p = synth.nodegraph_pair(0)
    g, gg = _graphs(fr, p, 1.0)
    T = np.repeat(np.eye(4)[None], 512, 0)
    prm = fr.register_params(3, "pt2pt", p.sigma, iters=2, w=p.w)
    st, rep = fr.fr_register_nodegraph(ctx.h, upload([p.model]), upload([p.obs]), gg, prm, T)
    ref = ng.register_nodegraph(g, p.model, None, p.obs, None, sigma=p.sigma, w=p.w, lam=1.0, iters=2)
    assert st == 0
    err = max(oracle.rotation_angle(T[k][:3, :3] @ ref[k][:3, :3].T) for k in range(512))
    assert err < 1e-4
    assert np.abs(T[:, :3, 3] - ref[:, :3, 3]).max() < 1e-4
