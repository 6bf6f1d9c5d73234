"""The autotuner on a GPU: it times each candidate setting on the caller's path, caches
the winner, and the winning plan computes the same gradient as the default plan."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_picks_a_candidate_and_caches_it(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_11962_amd as mop
    from paper_2501_11962_amd import autotune as A
    s = W.water_box(1002, seed=9, rc=1.0)
    N = 3
    R, _, _ = W.random_walk_path(s, N, 41)
    Rt = torch.from_numpy(R).cuda()
    ctx = mop.Context()
    cands = [dict(col_width=0.4, waves=4), dict(col_width=0.5, waves=2)]
    cache = str(tmp_path / "tune.json")
    seen = []
    best = A.autotune(ctx, s, Rt, candidates=cands, repeats=2, cache=cache, log=seen.append)
    assert best in cands
    assert len(seen) == len(cands)
    table = A.load_cache(cache)
    key = A.shape_key(s, N)
    assert table[key]["opts"] == best and len(table[key]["tried"]) == len(cands)
    # a second call is answered from the cache without timing anything
    seen.clear()
    assert A.autotune(ctx, s, Rt, candidates=cands, cache=cache, log=seen.append) == best
    assert not seen
    sysm = mop.System(ctx, s)
    G0, v0 = mop.veff_grad(mop.Plan(sysm, N), Rt)
    G1, v1 = mop.veff_grad(mop.Plan(sysm, N, **best), Rt)
    G0, G1 = G0.cpu().numpy(), G1.cpu().numpy()
    assert np.linalg.norm(G1 - G0) < 1e-5 * np.linalg.norm(G0)
    assert abs(float(v1[0]) - float(v0[0])) < 1e-6 * abs(float(v0[0]))
