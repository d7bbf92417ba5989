"""GPU: the autotuner picks the fastest measured leaf level / chunk width, and the operator
it picks computes the same product as any other choice (the H^2 operator depends on the
leaf level, so the check is against the oracle with the chosen parameters)."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_picks_a_measured_candidate(orc, tmp_path):
    import paper_1906_00785_amd as B
    import paper_1906_00785_amd.autotune as AT

    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=1, level=3)
    cache = str(tmp_path / "tune.json")
    res = AT.tune(s, q=4, eta=1.6, steps=5, cache=cache)
    timed = [r for r in res["table"] if "apply_us" in r]
    assert timed and res["apply_us"] == min(r["apply_us"] for r in timed)
    assert res["leaf_level"] in range(0, 4)
    # cached: the second call reads the file
    assert AT.tune(s, q=4, eta=1.6, steps=5, cache=cache) == res
    A = B.Operator(s, q=4, eta=1.6, leaf_level=res["leaf_level"], chunk_cols=res["chunk_cols"])
    So = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=1, level=3)
    Ho = orc.H2(So, q=4, eta=1.6, leaf=res["leaf_level"])
    x = W.random_vector(W.rng(0, 400), s.ndof)
    y = A.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    yo = Ho.apply(x)
    assert np.max(np.abs(y - yo)) <= 1e-11 * np.max(np.abs(yo))
