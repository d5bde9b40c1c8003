"""Precision form at N = 6: FP32 and split-BF16 operator products against the FP64 oracle.

The 3072-tetrahedron unit cube at N = 6 (1.03 M unknowns) with the rigid-box eigenmode:
single-rate AB3 from the exact history, relative L2 of all four fields against the oracle's
FP64 AB3 every 100 steps up to 500 (and against the closed form).  A 3-level two-layer mesh
at N = 6 checks the multi-rate path the same way over 100 local steps, and a checkpointed RTM
shot on it the characteristic image.  The measured errors are printed (pytest -s) and bounded:
fields FP32 <= 1e-5 and split-BF16 <= 1e-4 after 100 steps, images <= 1e-4 in both forms."""
import numpy as np
import pytest

from oracle import timestep as T
from oracle.mesh import BC_RIGID, BC_TRANSPARENT
from paper_1506_00907_amd import inputs as I
from tests.oracle_cases import case, eigenmode, oracle_shot

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(a, b):
    return float(np.linalg.norm((np.asarray(a, np.float64) - b).ravel()) / np.linalg.norm(b.ravel()))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


@pytest.fixture(scope="module")
def cube6():
    from paper_1506_00907_amd import dgrtm
    mm, rho, c, N = I.config_mesh("eigen_cube_n6")
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_RIGID).set_model(rho, c, 1).bind("cuda")
    m, op, lev, L, dtl = case("eigen_cube_n6", bc=BC_RIGID, n_levels=1)
    assert lm.dt_local == dtl
    return lm, op, dtl


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4)])
def test_eigenmode_n6_error_every_100_steps(cube6, precision, tol):
    from paper_1506_00907_amd import dgrtm
    lm, op, dtl = cube6
    M = op.m
    q0 = eigenmode(M, 0.0)
    h1, h2 = op.rhs(eigenmode(M, -dtl)), op.rhs(eigenmode(M, -2 * dtl))
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=500 * dtl, precision=precision))
    shot.set_state(dgrtm.SOURCE_FIELD, _dev(q0), _dev(h1), _dev(h2))
    qo, ho = q0, np.stack([h1, h2])
    e0 = np.sqrt(op.energy(q0))
    report = []
    for blk in range(5):
        shot.run(dgrtm.SOURCE_FIELD, 100)
        qo, ho = T.ab3(op, qo, dtl, 100, hist=ho, t0=blk * 100 * dtl)
        got = shot.get_state(dgrtm.SOURCE_FIELD).cpu().numpy()
        ex = eigenmode(M, (blk + 1) * 100 * dtl)
        report.append(((blk + 1) * 100, _rel(got, qo), float(np.sqrt(op.energy(got - ex)) / e0)))
    name = "FP32" if precision == 0 else "split-BF16"
    for st, e_or, e_cf in report:
        print(f"N=6 cube {name}: step {st}: rel L2 vs FP64 oracle {e_or:.3e}, vs closed form {e_cf:.3e}")
    assert report[0][1] <= tol
    assert all(r[1] <= 10 * tol for r in report)


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4)])
def test_multirate_n6_100_steps(precision, tol):
    from paper_1506_00907_amd import dgrtm
    name = "two_layer_small:4:4:3:6"
    mm, rho, c, N = I.config_mesh(name)
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, 3).bind("cuda")
    m, op, lev, L, dtl = case(name, bc=BC_TRANSPARENT, n_levels=3)
    x = op.m.x
    q0 = np.zeros((op.m.K, 4, op.ref.Np))
    q0[:, 0] = np.exp(-((x[..., 0] - 1) ** 2 + (x[..., 1] - 1) ** 2 + (x[..., 2] - 0.5) ** 2) / 0.05)
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=100 * dtl * 2 ** (L - 1), precision=precision))
    shot.set_state(dgrtm.SOURCE_FIELD, _dev(q0))
    ng = 100 // 2 ** (L - 1)
    shot.run(dgrtm.SOURCE_FIELD, ng)
    st = T.MRAB(op, lev, L, dtl)
    st.set_state(q0)
    for _ in range(ng):
        st.global_step()
    err = _rel(shot.get_state(dgrtm.SOURCE_FIELD).cpu().numpy(), st.q)
    print(f"N=6 two-layer 3-level MRAB {'FP32' if precision == 0 else 'split-BF16'}: "
          f"{ng * 2 ** (L - 1)} local steps: rel L2 vs FP64 oracle {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("precision", [0, 1])
def test_image_n6(precision):
    from paper_1506_00907_amd import dgrtm
    name = "two_layer_small:4:4:3:6"
    mm, rho, c, N = I.config_mesh(name)
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, 3).bind("cuda")
    m, op, lev, L, dtl = case(name, bc=BC_TRANSPARENT, n_levels=3)
    spec = I.rtm_shot(n_rec=4)
    spec.t_peak = 0.02
    ng = 16
    shot = dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=ng * dtl * 2 ** (L - 1), src=spec.src, f_peak=spec.f_peak,
                                         t_peak=spec.t_peak, rec=spec.rec, ckpt_interval=5, precision=precision))
    tr = shot.forward()
    shot.adjoint(tr, dgrtm.IMAGE_CHARACTERISTIC, (0.0, 0.0, 1.0), 0)
    img = shot.image().cpu().numpy()
    osh = oracle_shot(op, lev, L, dtl, ng, spec)
    osh.forward()
    img_ref = osh.adjoint(tr.cpu().numpy().astype(np.float64))
    err = _rel(img, img_ref)
    print(f"N=6 characteristic image, {ng} global steps, {'FP32' if precision == 0 else 'split-BF16'}: "
          f"rel L2 vs FP64 oracle {err:.3e}")
    assert err <= 1e-4
