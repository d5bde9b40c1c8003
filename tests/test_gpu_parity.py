"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP32 fields <= 1e-5 relative L2 after 100 steps, images <= 1e-4 relative L2;
one rhs application <= 2e-6 (a single FP32 operator evaluation)."""
import numpy as np
import pytest

from oracle import source as OS
from oracle import timestep as T
from oracle.mesh import BC_FREE, BC_RIGID, BC_TRANSPARENT, OMesh, local_dt, lts_levels
from oracle.rtm import COND_CHARACTERISTIC, COND_PRESSURE, Shot as OShot
from oracle.refelem import get_ref
from paper_1506_00907_amd import inputs as I
from tests.oracle_cases import case, eigenmode, oracle_shot

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def lib_mesh(name, bc, nl, face_bc=None, rho=None, c=None):
    from paper_1506_00907_amd import dgrtm
    mm, rho0, c0, N = I.config_mesh(name)
    rho = rho0 if rho is None else rho
    c = c0 if c is None else c
    m = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=bc, face_bc=face_bc).set_model(rho, c, n_levels_max=nl)
    return m.bind("cuda"), mm, rho, c, N


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


@pytest.mark.parametrize("name", ["two_layer_small:4:4:3:3", "two_layer_small:4:3:3:4", "two_layer_small:3:3:2:5",
                                  "two_layer_small:3:2:2:2", "two_layer_small:2:2:2:1"])
@pytest.mark.parametrize("reversed_time", [False, True])
def test_rhs_parity_mixed_boundaries(name, reversed_time):
    from paper_1506_00907_amd import dgrtm
    mm, rho, c, N = I.config_mesh(name)
    rng = np.random.default_rng(11)
    rho = rho * rng.uniform(0.8, 1.5, mm.K)
    bc = rng.choice([BC_RIGID, BC_TRANSPARENT, BC_FREE], size=(mm.K, 4)).astype(np.int8)
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, face_bc=bc).set_model(rho, c, n_levels_max=3).bind("cuda")
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=lm.dt_local))
    om = OMesh(get_ref(N), mm.verts, mm.etov, face_bc=bc)
    from oracle.dg import Operator
    op = Operator(om, rho, c)
    q = rng.standard_normal((mm.K, 4, lm.Np))
    got = shot.apply_rhs(dev(q), reversed_time=reversed_time).cpu().numpy()
    ref = op.rhs_reversed(q) if reversed_time else op.rhs(q)
    assert rel(got, ref) < 2e-6


def test_single_rate_ab3_eigenmode_100_steps():
    from paper_1506_00907_amd import dgrtm
    lm, mm, rho, c, N = lib_mesh("eigen_cube", BC_RIGID, 1)
    m, op, lev, L, dtl = case("eigen_cube", bc=BC_RIGID, n_levels=1)
    assert lm.dt_local == dtl and lm.L == 1
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=100 * dtl))
    M = op.m
    q0 = eigenmode(M, 0.0)
    h1, h2 = op.rhs(eigenmode(M, -dtl)), op.rhs(eigenmode(M, -2 * dtl))
    shot.set_state(dgrtm.SOURCE_FIELD, dev(q0), dev(h1), dev(h2))
    shot.run(dgrtm.SOURCE_FIELD, 100)
    got = shot.get_state(dgrtm.SOURCE_FIELD).cpu().numpy()
    ref, _ = T.ab3(op, q0, dtl, 100, hist=np.stack([h1, h2]))
    assert rel(got, ref) < 1e-5
    # and the closed form is met to the discretisation error
    e = np.sqrt(op.energy(got - eigenmode(M, 100 * dtl)) / op.energy(q0))
    assert e < 2e-4


def _oracle_shot(name, lev, L, dtl, op, n_global, spec):
    return oracle_shot(op, lev, L, dtl, n_global, spec)


@pytest.mark.parametrize("name,nl", [("two_layer_small:6:6:4:3", 3), ("two_layer_small:5:5:3:4", 3),
                                     ("two_layer_small:4:4:3:5", 3)])
def test_multirate_forward_fields_and_traces(name, nl):
    from paper_1506_00907_amd import dgrtm
    lm, mm, rho, c, N = lib_mesh(name, BC_TRANSPARENT, nl)
    m, op, lev, L, dtl = case(name, bc=BC_TRANSPARENT, n_levels=nl)
    assert L == lm.L and L >= 2
    spec = I.rtm_shot(n_rec=5)
    ng = 100 // (2 ** (L - 1)) + 1
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=ng * dtl * 2 ** (L - 1), src=spec.src, f_peak=spec.f_peak,
                                         t_peak=0.02, rec=spec.rec))
    assert shot.n_global == ng
    tr = shot.forward().cpu().numpy()
    q = shot.get_state(dgrtm.SOURCE_FIELD).cpu().numpy()
    spec.t_peak = 0.02
    osh = _oracle_shot(name, lev, L, dtl, op, ng, spec)
    tr_ref = osh.forward(keep=False)
    assert rel(q, osh.S_final) < 1e-5
    assert rel(tr, tr_ref) < 1e-5


@pytest.mark.parametrize("cond", [COND_CHARACTERISTIC, COND_PRESSURE])
@pytest.mark.parametrize("ckpt", [0, 3])
def test_rtm_image_parity(cond, ckpt):
    from paper_1506_00907_amd import dgrtm
    name = "two_layer_small:6:6:4:2"
    lm, mm, rho, c, N = lib_mesh(name, BC_TRANSPARENT, 3)
    m, op, lev, L, dtl = case(name, bc=BC_TRANSPARENT, n_levels=3)
    spec = I.rtm_shot(n_rec=4)
    spec.t_peak = 0.03
    ng = 30
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=ng * dtl * 2 ** (L - 1), src=spec.src, f_peak=spec.f_peak,
                                         t_peak=spec.t_peak, rec=spec.rec, ckpt_interval=ckpt))
    tr = shot.forward()
    shot.adjoint(tr, condition=cond, up=(0.0, 0.0, 1.0), g_image_start=4)
    img = shot.image().cpu().numpy()
    osh = _oracle_shot(name, lev, L, dtl, op, ng, spec)
    tr_ref = osh.forward(condition=cond)
    assert rel(tr.cpu().numpy(), tr_ref) < 1e-5
    img_ref = osh.adjoint(tr.cpu().numpy().astype(np.float64), condition=cond, g_image_start=4)
    assert rel(img, img_ref) < 1e-4


def _top_free_face_bc(mm, nx, ny):
    """Free surface (p = 0) on the faces in the top plane z = Lz, transparent elsewhere; faces
    numbered on the re-oriented element, as the library and the oracle both read them."""
    from oracle.mesh import orient
    from oracle.refelem import FACE_VERTS
    verts = np.asarray(mm.verts, dtype=np.float64)
    et = orient(verts, np.asarray(mm.etov, dtype=np.int64))
    bc = np.full((mm.K, 4), BC_TRANSPARENT, dtype=np.int8)
    for f, lv in enumerate(FACE_VERTS):
        on_top = np.all(np.abs(verts[et[:, list(lv)], 2] - mm.box[2]) < 1e-12, axis=1)
        bc[on_top, f] = BC_FREE
    assert (bc == BC_FREE).sum() == 2 * nx * ny      # two triangles per top cell
    return bc


@pytest.mark.parametrize("up", [(0.0, 0.0, 1.0), (0.5, 0.0, 0.8660254037844386)])
def test_free_surface_top_oblique_up_and_stacked_image(up):
    """A free-surface top boundary, a vertical or an oblique characteristic direction, and two
    shots stacked into one image through the accumulate form of dgrtm_image."""
    from oracle.dg import Operator
    from paper_1506_00907_amd import dgrtm
    name = "two_layer_small:6:6:4:2"
    mm, rho, c, N = I.config_mesh(name)
    bc = _top_free_face_bc(mm, 6, 6)
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, face_bc=bc).set_model(rho, c, n_levels_max=3).bind("cuda")
    om = OMesh(get_ref(N), mm.verts, mm.etov, face_bc=bc)
    op = Operator(om, rho, c)
    lev, L, dtl = lts_levels(local_dt(om.verts, om.etov, c, N), om.EToE, 3)
    assert L == lm.L and L >= 2
    ng = 30
    stack = torch.zeros((lm.K, lm.Np), dtype=torch.float64, device="cuda")
    imgs, refs = [], []
    for src_xy in [(0.7797, 1.0), (1.3, 0.6)]:
        spec = I.rtm_shot(src_xy=src_xy, n_rec=4)
        spec.t_peak = 0.03
        shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=ng * dtl * 2 ** (L - 1), src=spec.src, f_peak=spec.f_peak,
                                             t_peak=spec.t_peak, rec=spec.rec, ckpt_interval=4))
        tr = shot.forward()
        shot.adjoint(tr, condition=dgrtm.IMAGE_CHARACTERISTIC, up=up, g_image_start=4)
        imgs.append(shot.image().cpu().numpy())
        shot.image(out=stack, accumulate=True)
        osh = oracle_shot(op, lev, L, dtl, ng, spec)
        tr_ref = osh.forward(condition=COND_CHARACTERISTIC, up=up)
        assert rel(tr.cpu().numpy(), tr_ref) < 1e-5
        refs.append(osh.adjoint(tr.cpu().numpy().astype(np.float64), condition=COND_CHARACTERISTIC, up=up,
                                g_image_start=4))
        assert rel(imgs[-1], refs[-1]) < 1e-4
    stack = stack.cpu().numpy()
    assert np.array_equal(stack, imgs[0] + imgs[1])
    assert rel(stack, refs[0] + refs[1]) < 1e-4


def test_residual_fp64():
    from paper_1506_00907_amd import dgrtm
    lm, *_ = lib_mesh("two_layer_small:2:2:2:1", BC_TRANSPARENT, 1)
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=lm.dt_local))
    rng = np.random.default_rng(3)
    a = rng.standard_normal(100003).astype(np.float32)
    b = rng.standard_normal(100003).astype(np.float32)
    r = shot.residual(dev(a), dev(b))
    ref = np.sum((a.astype(np.float64) - b.astype(np.float64)) ** 2)
    assert abs(r - ref) < 1e-12 * ref


@pytest.mark.parametrize("name", ["two_layer_small:4:4:3:3", "two_layer_small:4:3:3:4", "two_layer_small:3:3:2:5"])
def test_rhs_parity_split_bf16(name):
    from paper_1506_00907_amd import dgrtm
    mm, rho, c, N = I.config_mesh(name)
    lm = dgrtm.Mesh(N, mm.verts, mm.etov).set_model(rho, c, n_levels_max=3).bind("cuda")
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=lm.dt_local, precision=dgrtm.SPLIT_BF16))
    from oracle.dg import Operator
    m, op, *_ = case(name)
    rng = np.random.default_rng(5)
    # a smooth field plus noise: the relevant case for error growth
    x = op.m.x
    q = np.stack([np.sin(2 * x[..., 0]) * np.cos(x[..., 1] + x[..., 2])] * 4, axis=1)
    q += 0.01 * rng.standard_normal(q.shape)
    got = shot.apply_rhs(dev(q)).cpu().numpy()
    err = rel(got, op.rhs(q))
    assert err < 1e-4, err


@pytest.mark.parametrize("name,nl", [("two_layer_small:5:5:3:4", 3), ("two_layer_small:4:4:3:5", 3)])
def test_split_bf16_forward_100_steps(name, nl):
    from paper_1506_00907_amd import dgrtm
    lm, mm, rho, c, N = lib_mesh(name, BC_TRANSPARENT, nl)
    m, op, lev, L, dtl = case(name, bc=BC_TRANSPARENT, n_levels=nl)
    spec = I.rtm_shot(n_rec=5)
    spec.t_peak = 0.02
    ng = 100 // (2 ** (L - 1)) + 1
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=ng * dtl * 2 ** (L - 1), src=spec.src, f_peak=spec.f_peak,
                                         t_peak=spec.t_peak, rec=spec.rec, precision=dgrtm.SPLIT_BF16))
    tr = shot.forward().cpu().numpy()
    q = shot.get_state(dgrtm.SOURCE_FIELD).cpu().numpy()
    osh = _oracle_shot(name, lev, L, dtl, op, ng, spec)
    tr_ref = osh.forward(keep=False)
    assert rel(q, osh.S_final) < 1e-4
    assert rel(tr, tr_ref) < 1e-4


@pytest.mark.parametrize("name,precision", [("two_layer_small:6:6:4:2", 1), ("two_layer_small:4:4:3:4", 1),
                                            ("two_layer_small:4:4:3:5", 0), ("two_layer_small:4:4:3:5", 1)])
def test_checkpointed_image(name, precision):
    """Checkpointed characteristic image (forward, segment recompute with records, backward with
    the image) against the oracle; at N = 5 in both forms."""
    from paper_1506_00907_amd import dgrtm
    lm, mm, rho, c, N = lib_mesh(name, BC_TRANSPARENT, 3)
    m, op, lev, L, dtl = case(name, bc=BC_TRANSPARENT, n_levels=3)
    spec = I.rtm_shot(n_rec=4)
    spec.t_peak = 0.03
    ng = 30
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=ng * dtl * 2 ** (L - 1), src=spec.src, f_peak=spec.f_peak,
                                         t_peak=spec.t_peak, rec=spec.rec, ckpt_interval=4,
                                         precision=precision))
    tr = shot.forward()
    shot.adjoint(tr, condition=COND_CHARACTERISTIC, up=(0.0, 0.0, 1.0), g_image_start=0)
    img = shot.image().cpu().numpy()
    osh = _oracle_shot(name, lev, L, dtl, op, ng, spec)
    tr_ref = osh.forward()
    assert rel(tr.cpu().numpy(), tr_ref) < (1e-5 if precision == 0 else 1e-4)
    img_ref = osh.adjoint(tr.cpu().numpy().astype(np.float64))
    assert rel(img, img_ref) < 1e-4


def test_batched_shots_match_alone():
    """Continuous batching: shots that join a running batch at different times give the same
    traces and image as each shot run alone (same kernels, per-slot state; target bitwise)."""
    from paper_1506_00907_amd import dgrtm
    name = "two_layer_small:5:5:3:3"
    lm, mm, rho, c, N = lib_mesh(name, BC_TRANSPARENT, 3)
    dtg = lm.dt_local * 2 ** (lm.L - 1)
    srcs = [(0.6, 0.9), (1.3, 1.1), (1.0, 0.5)]
    specs = []
    for x, y in srcs:
        sp = I.rtm_shot(src_xy=(x, y), n_rec=4)
        specs.append(dgrtm.ShotSpec(t_final=24 * dtg, src=sp.src, f_peak=15.0, t_peak=0.03, rec=sp.rec,
                                    ckpt_interval=5))
    alone = []
    for sp in specs:
        sh = dgrtm.Shot(lm, sp)
        tr = sh.forward()
        sh.adjoint(tr, condition=dgrtm.IMAGE_CHARACTERISTIC, up=(0, 0, 1), g_image_start=2)
        alone.append((tr.cpu().numpy(), sh.image().cpu().numpy()))
    shots = [dgrtm.Shot(lm, sp) for sp in specs]
    start = [0, 3, 11]                       # global step at which each request joins
    active = []
    tick = 0
    while True:
        for i, s0 in enumerate(start):
            if s0 == tick:
                shots[i].begin(None, dgrtm.IMAGE_CHARACTERISTIC, (0, 0, 1), 2)
                active.append(shots[i])
        live = [s for s in active if s.state()[0] != dgrtm.PHASE_DONE]
        if not live and tick > max(start):
            break
        if live:
            dgrtm.step_shots(live, 1)
        tick += 1
    for sh, (tr_a, img_a) in zip(shots, alone):
        tr_b = sh.traces().cpu().numpy()
        img_b = sh.image().cpu().numpy()
        assert np.array_equal(tr_a, tr_b)
        assert rel(img_b, img_a) <= 1e-6
    # the shot that joined last, as it came out of the batch, against the oracle
    m, op, lev, L, dtl = case(name, bc=BC_TRANSPARENT, n_levels=3)
    sp = I.rtm_shot(src_xy=srcs[2], n_rec=4)
    sp.t_peak = 0.03
    osh = _oracle_shot(name, lev, L, dtl, op, 24, sp)
    tr_ref = osh.forward()
    tr_b = shots[2].traces().cpu().numpy()
    assert rel(tr_b, tr_ref) < 1e-5
    img_ref = osh.adjoint(tr_b.astype(np.float64), g_image_start=2)
    assert rel(shots[2].image().cpu().numpy(), img_ref) < 1e-4
