"""Full-size checks on the 201 600-element two-layer mesh (N = 4) in the launch configuration the
benchmark times.  Launches with at least three tiles per wavefront hand tiles out from a per-slot
counter and stagger the starts of their wavefronts; no small mesh triggers that, so these tests
run the benchmark's mesh:

- the right-hand side against the FP64 oracle on sampled elements (the oracle evaluates them one
  by one from the same state), in FP32 and in split-BF16;
- a whole checkpointed shot of three global steps against the oracle's shot on the whole mesh;
- a whole shot (forward, checkpointed recompute, backward with image) with the counter hand-out
  against the same shot with every wavefront on fixed tiles: bit for bit;
- two shots sharing every launch (two slots, two counters) against each shot alone: bit for bit;
- the same fixed-tile comparison for the N >= 5 kernel on an 80k-element N = 5 mesh;
- the rhs on the 4.1M-element, 4-level mesh of the largest shot, the 786k-element N = 5 serving
  mesh and the 200k-element mesh at N = 6 against the oracle on sampled elements (the oracle set
  up on the sampled elements and their face neighbours only).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAME = "rtm_200k"


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def big():
    from paper_1506_00907_amd import dgrtm, inputs as I
    mm, rho, c, N = I.config_mesh(NAME)
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, 3).bind("cuda")
    assert lm.K == 201600 and lm.L == 3
    return lm, mm, rho, c, N


def _spec(mm, src_xy, n_global, lm, ckpt_interval):
    from paper_1506_00907_amd import dgrtm, inputs as I
    s = I.rtm_shot(box=mm.box, src_xy=src_xy, n_rec=20, t_final=1.0)
    t_final = n_global * lm.dt_local * 2 ** (lm.L - 1)
    # an early pulse, so that the short run carries a real wavefield
    return dgrtm.ShotSpec(t_final=t_final, src=s.src, f_peak=s.f_peak, t_peak=0.002, rec=s.rec,
                          ckpt_interval=ckpt_interval)


def _alone(lm, spec):
    from paper_1506_00907_amd import dgrtm
    sh = dgrtm.Shot(lm, spec)
    tr = sh.forward()
    q = sh.get_state(dgrtm.SOURCE_FIELD).cpu().numpy()
    sh.adjoint(tr, dgrtm.IMAGE_CHARACTERISTIC, (0.0, 0.0, 1.0), 0)
    img = sh.image().cpu().numpy()
    return tr.cpu().numpy(), q, img


@pytest.fixture(scope="module")
def big_oracle(big):
    """The oracle's operator and LTS levels on the whole mesh."""
    from oracle.dg import Operator
    from oracle.mesh import BC_TRANSPARENT, OMesh, local_dt, lts_levels
    from oracle.refelem import get_ref
    lm, mm, rho, c, N = big
    om = OMesh(get_ref(N), mm.verts, mm.etov, bc_default=BC_TRANSPARENT)
    op = Operator(om, rho, c)
    lev, L, dtl = lts_levels(local_dt(om.verts, om.etov, c, N), om.EToE, 3)
    return om, op, lev, L, dtl


@pytest.mark.parametrize("reversed_time,precision", [(False, 0), (True, 0), (False, 1), (True, 1)])
def test_full_size_rhs_sampled_vs_oracle(big, big_oracle, reversed_time, precision):
    from paper_1506_00907_amd import dgrtm
    lm, mm, rho, c, N = big
    om, op = big_oracle[:2]
    rng = np.random.default_rng(21)
    x = om.x
    smooth = np.sin(3.0 * x[..., 0]) * np.cos(2.0 * x[..., 1] + x[..., 2])
    q = np.stack([smooth, 0.5 * smooth, -smooth, 0.25 * smooth], axis=1)
    q += 0.01 * rng.standard_normal(q.shape)
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=lm.dt_local, precision=precision))
    got = shot.apply_rhs(torch.from_numpy(q.astype(np.float32)).cuda(), reversed_time=reversed_time)
    got = got.cpu().numpy()
    el = np.sort(rng.choice(lm.K, 4000, replace=False))
    ref = op.rhs_reversed(q, elems=el) if reversed_time else op.rhs(q, elems=el)
    # one FP32 operator evaluation; split-BF16 products (hi*hi + hi*lo + lo*hi) on a smooth field
    assert rel(got[el], ref) < (2e-6 if precision == 0 else 1e-4)


def test_full_size_shot_vs_oracle(big, big_oracle):
    """A whole checkpointed shot (forward, recompute, backward with the image) on the whole mesh,
    three global steps, against the oracle's shot: traces, final source field and image."""
    from oracle.rtm import COND_CHARACTERISTIC
    from paper_1506_00907_amd import dgrtm
    from tests.oracle_cases import oracle_shot
    lm, mm, rho, c, N = big
    om, op, lev, L, dtl = big_oracle
    assert L == lm.L and dtl == lm.dt_local
    ng = 3
    spec = _spec(mm, (0.7797, 1.0), ng, lm, ckpt_interval=2)
    # a receiver beside the source, so that the traces and the image are not zero this early
    spec.rec = np.vstack([spec.rec, spec.src + np.array([0.001, 0.001, -0.002])])
    sh = dgrtm.Shot(lm, spec)
    tr = sh.forward()
    q = sh.get_state(dgrtm.SOURCE_FIELD).cpu().numpy()
    sh.adjoint(tr, dgrtm.IMAGE_CHARACTERISTIC, (0.0, 0.0, 1.0), 0)
    img = sh.image().cpu().numpy()
    osh = oracle_shot(op, lev, L, dtl, ng, spec)
    tr_ref = osh.forward(condition=COND_CHARACTERISTIC)
    assert np.abs(tr_ref).max() > 0
    assert rel(tr.cpu().numpy(), tr_ref) < 1e-5
    assert rel(q, osh.S_final) < 1e-5
    img_ref = osh.adjoint(tr.cpu().numpy().astype(np.float64), condition=COND_CHARACTERISTIC, g_image_start=0)
    assert np.abs(img_ref).max() > 0
    assert rel(img, img_ref) < 1e-4


def test_full_size_counter_handout_matches_fixed_tiles(big):
    lm, mm, rho, c, N = big
    spec = _spec(mm, (0.7797, 1.0), 27, lm, ckpt_interval=8)   # 4 segments in the adjoint
    lm.set_launch_cap(0)
    a = _alone(lm, spec)
    try:
        lm.set_launch_cap(1 << 30)    # one work-group per tile group: fixed tiles, no stagger
        b = _alone(lm, spec)
    finally:
        lm.set_launch_cap(0)
    assert np.abs(a[0]).max() > 0 and np.abs(a[2]).max() > 0
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_full_size_two_slots_match_alone(big):
    from paper_1506_00907_amd import dgrtm
    lm, mm, rho, c, N = big
    specs = [_spec(mm, (0.7797, 1.0), 19, lm, 6), _spec(mm, (1.3, 0.6), 19, lm, 6)]
    alone = [_alone(lm, s) for s in specs]
    shots = [dgrtm.Shot(lm, s) for s in specs]
    for sh in shots:
        sh.begin(None, dgrtm.IMAGE_CHARACTERISTIC, (0.0, 0.0, 1.0), 0)
    for _ in range(10000):
        if all(sh.state()[0] == dgrtm.PHASE_DONE for sh in shots):
            break
        dgrtm.step_shots(shots, 1)
    for sh, (tr, _, img) in zip(shots, alone):
        assert sh.state()[0] == dgrtm.PHASE_DONE
        assert np.array_equal(sh.traces().cpu().numpy(), tr)
        assert np.array_equal(sh.image().cpu().numpy(), img)


def test_n5_counter_handout_matches_fixed_tiles():
    from paper_1506_00907_amd import dgrtm, inputs as I
    mm, rho, c, N = I.config_mesh("two_layer_small:28:28:17:5")
    assert N == 5 and mm.K // 16 >= 3 * 4 * 256   # the full-prefix launches hand tiles out
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, 3).bind("cuda")
    spec = _spec(mm, (1.0, 1.0), 13, lm, ckpt_interval=4)
    a = _alone(lm, spec)
    try:
        lm.set_launch_cap(1 << 30)
        b = _alone(lm, spec)
    finally:
        lm.set_launch_cap(0)
    assert np.abs(a[0]).max() > 0 and np.abs(a[2]).max() > 0
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


_LARGE = {}


def _large(name, levels):
    """One large bound mesh at a time (kept across the cases that use it) and a seeded state."""
    from paper_1506_00907_amd import dgrtm, inputs as I
    if name not in _LARGE:
        _LARGE.clear()
        mm, rho, c, N = I.config_mesh(name)
        lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, levels).bind("cuda")
        assert lm.L == levels
        print(f"{name} bound: {lm.K} elements, N = {N}, {lm.L} levels", flush=True)
        q = torch.randn((lm.K, 4, lm.Np), generator=torch.Generator().manual_seed(7), dtype=torch.float32)
        _LARGE[name] = (lm, mm, rho, c, N, q)
    return _LARGE[name]


# the largest shot's 4.1M-element 4-level mesh, the 786k-element N = 5 serving mesh, and the
# 200k-element mesh at N = 6 (the precision study), each in both forms
LARGE_CASES = [(name, levels, rev, prec) for name, levels in (("big_4m", 4), ("srv_800k", 3), ("rtm_200k_n6", 3))
               for rev, prec in ((False, 0), (True, 0), (False, 1))]


@pytest.mark.parametrize("name,levels,reversed_time,precision", LARGE_CASES)
def test_large_mesh_rhs_sampled_vs_oracle(name, levels, reversed_time, precision):
    from paper_1506_00907_amd import dgrtm
    from tests.oracle_cases import neighbourhood_operator
    lm, mm, rho, c, N, q = _large(name, levels)
    rng = np.random.default_rng(31 + precision)
    el = np.sort(rng.choice(lm.K, 2000, replace=False))
    op, sub, loc = neighbourhood_operator(N, mm.verts, mm.etov, rho, c, el)
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=lm.dt_local, precision=precision))
    got = shot.apply_rhs(q.cuda(), reversed_time=reversed_time)[torch.from_numpy(el).cuda()].cpu().numpy()
    qs = q.numpy()[sub].astype(np.float64)
    ref = op.rhs_reversed(qs, elems=loc) if reversed_time else op.rhs(qs, elems=loc)
    err = rel(got, ref)
    print(f"{name} rhs, reversed={reversed_time}, precision={precision}: rel L2 {err:.3e}", flush=True)
    assert err < (2e-6 if precision == 0 else 1e-4)


def _progress(msg):
    # long oracle runs report their steps on the real stderr (pytest captures sys.stderr)
    import sys
    print(f"[fullsize] {msg}", file=sys.__stderr__, flush=True)


def _whole_shot_both_forms(name, levels, ng, ckpt):
    """A whole checkpointed shot (forward, recompute, backward with the characteristic image) on
    the whole mesh, in FP32 and in split-BF16, against one oracle shot.  Both forms and the
    oracle's backward run take the oracle's own traces (rounded to FP32) as the data, so the
    oracle runs once."""
    from oracle.dg import Operator
    from oracle.mesh import BC_TRANSPARENT, OMesh, local_dt, lts_levels
    from oracle.refelem import get_ref
    from oracle.rtm import COND_CHARACTERISTIC
    from paper_1506_00907_amd import dgrtm, inputs as I
    from tests.oracle_cases import oracle_shot
    mm, rho, c, N = I.config_mesh(name)
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, levels).bind("cuda")
    assert lm.K // 16 >= 3 * 4 * 256    # the full-prefix launches hand tiles out from the counter
    _progress(f"{name}: oracle set-up ({lm.K} elements, N = {N})")
    om = OMesh(get_ref(N), mm.verts, mm.etov, bc_default=BC_TRANSPARENT)
    op = Operator(om, rho, c)
    lev, L, dtl = lts_levels(local_dt(om.verts, om.etov, c, N), om.EToE, levels)
    assert L == lm.L and dtl == lm.dt_local
    spec = _spec(mm, (0.7797, 1.0), ng, lm, ckpt_interval=ckpt)
    spec.rec = np.vstack([spec.rec, spec.src + np.array([0.001, 0.001, -0.002])])
    osh = oracle_shot(op, lev, L, dtl, ng, spec)
    _progress(f"{name}: oracle forward")
    tr_ref = osh.forward(condition=COND_CHARACTERISTIC)
    data = tr_ref.astype(np.float32)
    _progress(f"{name}: oracle backward with image")
    img_ref = osh.adjoint(data.astype(np.float64), condition=COND_CHARACTERISTIC, g_image_start=0)
    assert np.abs(tr_ref).max() > 0 and np.abs(img_ref).max() > 0
    out = {}
    for prec, tol in ((dgrtm.FP32, 1e-5), (dgrtm.SPLIT_BF16, 1e-4)):
        spec.precision = prec
        sh = dgrtm.Shot(lm, spec)
        tr = sh.forward().cpu().numpy()
        q = sh.get_state(dgrtm.SOURCE_FIELD).cpu().numpy()
        sh.adjoint(torch.from_numpy(data).cuda(), dgrtm.IMAGE_CHARACTERISTIC, (0.0, 0.0, 1.0), 0)
        img = sh.image().cpu().numpy()
        out[prec] = (rel(tr, tr_ref), rel(q, osh.S_final), rel(img, img_ref))
        _progress(f"{name} precision {prec}: traces {out[prec][0]:.2e}, source field {out[prec][1]:.2e}, "
                  f"image {out[prec][2]:.2e}")
        assert out[prec][0] < tol and out[prec][1] < tol
        assert out[prec][2] < 1e-4
        del sh
    return out


def test_n5_whole_shot_vs_oracle():
    """The N >= 5 kernel (N = 5: operators in LDS) with counter hand-out, every step mode, both
    forms, against the oracle on an 80k-element mesh."""
    _whole_shot_both_forms("two_layer_small:28:28:17:5", 3, 3, 2)


def test_n6_whole_shot_vs_oracle():
    """The N = 6 kernel (operators through the caches), both forms, on the 201 600-element mesh of
    the precision study, against the oracle on the whole mesh."""
    _whole_shot_both_forms("rtm_200k_n6", 3, 2, 1)
