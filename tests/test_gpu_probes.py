"""Measurement entry points: the build's record counts and stage times, and the roofline probes."""
import numpy as np
import pytest

import synth
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


def test_records_and_stage_times(fr, ctx):
    # a 640x480 range-image frame merges most incidences into runs; a cloud in no order merges few
    p = synth.depth_pair(3)
    q = synth.ellipsoid_pair(1, m=3000)
    for obs, normals, feat, V, lo, hi in [(p.obs, p.obs_n, 6, 7, 0.1, 0.4), (q.obs, None, 3, 4, 0.9, 1.0)]:
        sig = p.sigma if feat == 6 else q.sigma
        lat = fr.Lattice(ctx, upload([obs], [normals] if normals is not None else None),
                         fr.lattice_params(feat, V, sig, 0.5))
        inc, part = fr.fr_lattice_records(lat.h)
        assert inc == (feat + 1) * len(obs)
        assert lo * inc <= part <= hi * inc, (feat, part / inc)
        t = fr.fr_lattice_build_times(lat.h)
        assert len(t) == 4 and all(x >= 0.0 for x in t) and sum(t) > 0.0
        lat.close()


def test_probes_report_positive_rates(fr, ctx):
    scat = fr.fr_probe_atomics(ctx.h, 1 << 20, 1 << 24, True)
    pack = fr.fr_probe_atomics(ctx.h, 1 << 20, 1 << 24, False)
    assert scat > 1e8 and pack > 1e8
    l1 = fr.fr_probe_lines(ctx.h, 1, 2 << 20)
    l8 = fr.fr_probe_lines(ctx.h, 8, 2 << 20)
    assert l1 > 1e9 and l8 > 1e9
    print(f"[probes] atomics scattered {scat:.3g}/s packed {pack:.3g}/s; L2 lines 1 lane {l1:.3g}/s, 8 lanes "
          f"{l8:.3g}/s", flush=True)
    with pytest.raises(fr.FRError):
        fr.fr_probe_atomics(ctx.h, 1 << 20, 3 << 20, True)       # not a power of two
    with pytest.raises(fr.FRError):
        fr.fr_probe_lines(ctx.h, 3, 2 << 20)                     # lanes per line not in {1, 2, 4, 8}
