"""End-to-end serving on the GPU: requests on two meshes served by continuous batching give
the same traces and images as the same requests served one at a time."""
import copy

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_serving_mix_equals_alone():
    from paper_1506_00907_amd import serving as S
    meshes = ["two_layer_small:5:5:3:3", "two_layer_small:4:4:3:4"]
    pools = {m: S.MeshSlotPool(m, n_rec=4) for m in meshes}
    reqs = S.make_requests(6, 200.0, meshes, t_final=0.01, seed=3)
    seq, bat = {}, {}
    rs = S.serve_sequential(pools, copy.deepcopy(reqs), results=seq)
    rb = S.serve_batched(pools, copy.deepcopy(reqs), hbm_budget=8 * 2 ** 30, max_slots=4, steps_per_tick=3,
                         results=bat)
    assert set(seq) == set(bat) == set(range(6))
    for rid in seq:
        (ta, ia), (tb, ib) = seq[rid], bat[rid]
        assert np.array_equal(ta, tb)
        assert np.linalg.norm(ia - ib) <= 1e-6 * np.linalg.norm(ia)
    for r in (rs, rb):
        s = r.summary()
        assert s["shots"] == 6 and s["latency_p99_s"] >= s["latency_p50_s"] > 0
