"""Degenerate cases of the HIP path against the FP64 oracle (through the C ABI):

- a mesh of one tetrahedron (a single padded tile, every face a boundary, given with negative
  orientation so the library re-orients it), N = 1..6, both time directions;
- the shortest shots: one and two global steps, with a checkpoint interval longer than the run,
  and with boundary-trace replay (whose start history then reaches back before t = 0);
- a one-tetrahedron shot with boundary-trace replay (every face replayed), N = 1..6;
- a shot without receivers (no traces, a zero image, the same source field as with receivers);
- source and receiver points outside the mesh (reported, nothing launched).
"""
import numpy as np
import pytest

from oracle.dg import Operator
from oracle.mesh import BC_FREE, BC_RIGID, BC_TRANSPARENT, OMesh, local_dt, lts_levels
from oracle.refelem import get_ref
from oracle.rtm import COND_CHARACTERISTIC
from paper_1506_00907_amd import inputs as I
from tests.oracle_cases import case, oracle_shot

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("reversed_time", [False, True])
def test_single_tetrahedron_rhs(N, reversed_time):
    from paper_1506_00907_amd import dgrtm
    verts = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1], [0.1, 0.2, 1.1]])
    etov = np.array([[0, 2, 1, 3]], dtype=np.int64)          # negative volume as given
    bc = np.array([[BC_RIGID, BC_TRANSPARENT, BC_FREE, BC_TRANSPARENT]], dtype=np.int8)
    rho, c = np.array([1.7]), np.array([2.3])
    lm = dgrtm.Mesh(N, verts, etov, face_bc=bc).set_model(rho, c, n_levels_max=3).bind("cuda")
    assert lm.K == 1 and lm.L == 1
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=lm.dt_local))
    op = Operator(OMesh(get_ref(N), verts, etov, face_bc=bc), rho, c)
    q = np.random.default_rng(N).standard_normal((1, 4, lm.Np))
    got = shot.apply_rhs(torch.from_numpy(q.astype(np.float32)).cuda(), reversed_time=reversed_time)
    ref = op.rhs_reversed(q) if reversed_time else op.rhs(q)
    assert rel(got.cpu().numpy(), ref) < 2e-6


@pytest.mark.parametrize("ng,ckpt,storage", [(1, 0, 0), (1, 5, 0), (2, 5, 0), (1, 0, 1), (2, 0, 1), (3, 0, 1)])
def test_shortest_shots_image(ng, ckpt, storage):
    from paper_1506_00907_amd import dgrtm
    name = "two_layer_small:6:6:4:2"
    mm, rho, c, N = I.config_mesh(name)
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, 3).bind("cuda")
    m, op, lev, L, dtl = case(name, bc=BC_TRANSPARENT, n_levels=3)
    assert L == lm.L
    # the source beside a receiver, an early pulse: the traces are not zero from the first step
    spec = I.rtm_shot(src_xy=(0.75, 0.75), n_rec=4)
    spec.t_peak = 0.002
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=ng * dtl * 2 ** (L - 1), src=spec.src, f_peak=spec.f_peak,
                                         t_peak=spec.t_peak, rec=spec.rec, ckpt_interval=ckpt, storage=storage))
    assert shot.n_global == ng
    tr = shot.forward()
    assert tr.shape == (16, ng + 1)
    shot.adjoint(tr, condition=dgrtm.IMAGE_CHARACTERISTIC, up=(0.0, 0.0, 1.0), g_image_start=0)
    img = shot.image().cpu().numpy()
    osh = oracle_shot(op, lev, L, dtl, ng, spec)
    tr_ref = osh.forward(condition=COND_CHARACTERISTIC, record_boundary=bool(storage))
    assert np.abs(tr_ref[:, -1]).max() > 0
    assert rel(tr.cpu().numpy(), tr_ref) < 1e-5
    run = osh.adjoint_replay if storage else osh.adjoint
    img_ref = run(tr.cpu().numpy().astype(np.float64), condition=COND_CHARACTERISTIC, g_image_start=0)
    assert np.abs(img_ref).max() > 0
    assert rel(img, img_ref) < 1e-4
    if storage:
        assert rel(shot.get_state(dgrtm.SOURCE_FIELD).cpu().numpy(), osh.S_back) < 1e-5


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_single_tetrahedron_replay_shot(N):
    """One tetrahedron with every face a boundary (rigid, transparent, free): the backward source
    run takes the exterior state of all four faces from the record."""
    from paper_1506_00907_amd import dgrtm
    verts = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1], [0.1, 0.2, 1.1]])
    etov = np.array([[0, 2, 1, 3]], dtype=np.int64)
    bc = np.array([[BC_RIGID, BC_TRANSPARENT, BC_FREE, BC_TRANSPARENT]], dtype=np.int8)
    rho, c = np.array([1.7]), np.array([2.3])
    lm = dgrtm.Mesh(N, verts, etov, face_bc=bc).set_model(rho, c, n_levels_max=3).bind("cuda")
    src = np.array([0.3, 0.3, 0.3])
    rec = np.array([[0.25, 0.3, 0.35]])
    ng = 12
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=ng * lm.dt_local, src=src, f_peak=15.0, t_peak=2 * lm.dt_local,
                                         rec=rec, storage=dgrtm.STORE_BOUNDARY))
    tr = shot.forward()
    shot.adjoint(tr, condition=dgrtm.IMAGE_CHARACTERISTIC, up=(0.0, 0.0, 1.0), g_image_start=0)
    img = shot.image().cpu().numpy()
    om = OMesh(get_ref(N), verts, etov, face_bc=bc)
    op = Operator(om, rho, c)
    lev, L, dtl = lts_levels(local_dt(om.verts, om.etov, c, N), om.EToE, 3)
    from tests.oracle_cases import oracle_shot as osf

    class Spec:
        pass
    sp = Spec()
    sp.src, sp.f_peak, sp.t_peak, sp.rec = src, 15.0, 2 * lm.dt_local, rec
    osh = osf(op, lev, L, dtl, ng, sp)
    tr_ref = osh.forward(condition=COND_CHARACTERISTIC, record_boundary=True)
    assert rel(tr.cpu().numpy(), tr_ref) < 1e-5
    img_ref = osh.adjoint_replay(tr.cpu().numpy().astype(np.float64), condition=COND_CHARACTERISTIC)
    assert rel(img, img_ref) < 1e-4
    assert rel(shot.get_state(dgrtm.SOURCE_FIELD).cpu().numpy(), osh.S_back) < 1e-5


def test_shot_without_receivers():
    from paper_1506_00907_amd import dgrtm
    name = "two_layer_small:4:4:3:3"
    mm, rho, c, N = I.config_mesh(name)
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, 3).bind("cuda")
    spec = I.rtm_shot(n_rec=3)
    t_final = 9 * lm.dt_local * 2 ** (lm.L - 1)
    kw = dict(t_final=t_final, src=spec.src, f_peak=spec.f_peak, t_peak=0.01, ckpt_interval=4)
    bare = dgrtm.Shot(lm, dgrtm.ShotSpec(**kw))
    assert bare.n_rec == 0 and bare.forward() is None
    q_bare = bare.get_state(dgrtm.SOURCE_FIELD).cpu().numpy()
    bare.adjoint(None, condition=dgrtm.IMAGE_CHARACTERISTIC, up=(0.0, 0.0, 1.0), g_image_start=0)
    assert np.all(bare.image().cpu().numpy() == 0.0)
    full = dgrtm.Shot(lm, dgrtm.ShotSpec(rec=spec.rec, **kw))
    full.forward()
    q_full = full.get_state(dgrtm.SOURCE_FIELD).cpu().numpy()
    assert np.abs(q_full).max() > 0 and np.array_equal(q_bare, q_full)


def test_points_outside_the_mesh_are_reported():
    from paper_1506_00907_amd import dgrtm
    mm, rho, c, N = I.config_mesh("two_layer_small:2:2:2:1")
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, 3).bind("cuda")
    inside = np.array([1.0, 1.0, 0.5])
    with pytest.raises(dgrtm.DgrtmError, match="outside the mesh"):
        dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=0.01, src=np.array([1.0, 1.0, 1.5])))
    with pytest.raises(dgrtm.DgrtmError, match="outside the mesh"):
        dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=0.01, src=inside, rec=np.array([[0.5, 0.5, 0.9], [2.5, 0.5, 0.9]])))
    sh = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=0.01, src=inside, rec=np.array([[0.5, 0.5, 0.9]])))
    assert sh.n_rec == 1
