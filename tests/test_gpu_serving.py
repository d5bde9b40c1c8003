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


def test_outputs_ordered_against_a_busy_mesh_stream():
    """A shot's image and traces read from the caller's stream while the mesh's own stream
    still holds queued steps of another shot must come back complete."""
    from paper_1506_00907_amd import dgrtm, serving as S
    pool = S.MeshSlotPool("two_layer_small:4:4:3:4", n_rec=4)
    reqs = S.make_requests(2, 200.0, [pool.name], t_final=0.02, seed=5)
    with torch.cuda.stream(pool.stream):
        a = dgrtm.Shot(pool.mesh, pool.spec(reqs[0]))
        tr = a.forward()
        a.adjoint(tr, dgrtm.IMAGE_CHARACTERISTIC, (0.0, 0.0, 1.0), 0)
        want_img = a.image().cpu().numpy()
        want_tr = a.traces().cpu().numpy()
        b = pool.new_shot(reqs[1])
        dgrtm.step_shots([b], 2 * b.n_global)          # queued on the mesh stream only
    got_img = a.image().cpu().numpy()                  # caller's (default) stream
    got_tr = a.traces().cpu().numpy()
    assert np.linalg.norm(want_img) > 0
    assert np.array_equal(got_img, want_img)
    assert np.array_equal(got_tr, want_tr)
    pool.sync()


def test_meshes_do_not_wait_for_each_other():
    """A long tick queued on one pool, then a short tick on another: the short one finishes first.
    (If a pool's tick waited for the work already queued on another pool's stream, it would end
    after the long one.)"""
    from paper_1506_00907_amd import dgrtm, serving as S
    long_pool = S.MeshSlotPool("two_layer_small:10:10:6:4", n_rec=4)
    short_pool = S.MeshSlotPool("two_layer_small:3:3:2:2", n_rec=4)
    req = S.Request(0, long_pool.name, (1.0, 1.0), 15.0, 0.0, 0.2)
    a = long_pool.new_shot(req)
    b = short_pool.new_shot(S.Request(1, short_pool.name, (1.0, 1.0), 15.0, 0.0, 0.2))
    torch.cuda.synchronize()
    ref = torch.cuda.Event(enable_timing=True)
    ref.record()
    torch.cuda.synchronize()
    ends = []
    for pool, shot, n in ((long_pool, a, 40), (short_pool, b, 1)):
        pool.step([shot], n)
        e = torch.cuda.Event(enable_timing=True)
        e.record(pool.stream)
        ends.append(e)
    torch.cuda.synchronize()
    t_long, t_short = (ref.elapsed_time(e) for e in ends)
    print(f"long tick ends at {t_long:.3f} ms, short tick at {t_short:.3f} ms", flush=True)
    assert a.state()[1] == 40 and b.state()[1] == 1
    assert t_short < 0.5 * t_long
