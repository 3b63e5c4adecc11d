"""Writes nodegraph_blob100k_oracle.npz: oracle node transforms of the node-graph workload (100k-point blob,
512 nodes, seed 0, sigma 0.02, w 0.1, lambda 1, 20 EM iterations from the identity) after iterations 10,
11, 19 and 20.  Calls only the oracle and the seeded generator:

    python tests/golden/make_nodegraph_states.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import nodegraph as ng  # noqa: E402

KEEP = (10, 11, 19, 20)


def main():
    p = synth.nodegraph_pair(0)
    e = p.extra
    g = ng.Graph(e["nodes"], e["skin_idx"], e["skin_w"], e["edges"])
    hist = []
    ng.register_nodegraph(g, p.model, None, p.obs, None, sigma=p.sigma, w=p.w, lam=1.0, iters=max(KEEP),
                          history=hist)
    out = {f"T{k}": hist[k - 1]["T"][:, :3, :4].copy() for k in KEEP}
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "nodegraph_blob100k_oracle.npz"),
                        **out)


if __name__ == "__main__":
    main()
