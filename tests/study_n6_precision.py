"""Precision study of the two forms at N = 6 on the 201 600-element two-layer mesh (the precision
configuration): relative L2 error of the source field against the FP64 oracle every 5 global
steps (20 local steps) up to 25 global steps (100 local steps), and of the characteristic image
of a checkpointed shot of those 25 global steps.

Not collected by default (the oracle needs several minutes for the whole mesh): run it by name,
python -m pytest tests/study_n6_precision.py -m gpu -s.  the design doc quotes its output."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a, np.float64) - b).ravel()) / np.linalg.norm(np.ravel(b)))


def _say(msg):
    import sys
    print(f"[study] {msg}", file=sys.__stderr__, flush=True)


def test_n6_precision_study():
    from oracle.dg import Operator
    from oracle.mesh import BC_TRANSPARENT, OMesh, local_dt, lts_levels
    from oracle.refelem import get_ref
    from oracle.rtm import COND_CHARACTERISTIC
    from paper_1506_00907_amd import dgrtm, inputs as I
    from tests.oracle_cases import oracle_shot
    mm, rho, c, N = I.config_mesh("rtm_200k_n6")
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, 3).bind("cuda")
    _say("oracle set-up")
    om = OMesh(get_ref(N), mm.verts, mm.etov, bc_default=BC_TRANSPARENT)
    op = Operator(om, rho, c)
    lev, L, dtl = lts_levels(local_dt(om.verts, om.etov, c, N), om.EToE, 3)
    assert L == lm.L and dtl == lm.dt_local
    every, ng = 5, 25
    s = I.rtm_shot(box=mm.box, src_xy=(0.7797, 1.0), n_rec=20)
    s.t_peak = 0.004                     # an early pulse, so that 25 global steps carry a wavefield
    s.rec = np.vstack([s.rec, s.src + np.array([0.001, 0.001, -0.002])])
    # the oracle's shot, with its source field every 5 global steps
    osh = oracle_shot(op, lev, L, dtl, ng, s)
    _say("oracle forward")
    tr_ref = osh.forward(condition=COND_CHARACTERISTIC, snap_every=every,
                         progress=lambda g: _say(f"oracle forward: global step {g} of {ng}"))
    states = osh.snaps
    data = tr_ref.astype(np.float32)
    img_ref = osh.adjoint(data.astype(np.float64), condition=COND_CHARACTERISTIC,
                          progress=lambda g: _say(f"oracle backward with image: global step {g} of {ng}"))
    for prec, name in ((dgrtm.FP32, "FP32"), (dgrtm.SPLIT_BF16, "split-BF16")):
        spec = dgrtm.ShotSpec(t_final=ng * lm.dt_local * 2 ** (lm.L - 1), src=s.src, f_peak=s.f_peak, t_peak=s.t_peak,
                              rec=s.rec, precision=prec)
        sh = dgrtm.Shot(lm, spec)
        errs = []
        sh.set_state(dgrtm.SOURCE_FIELD, None)
        for i in range(ng // every):
            sh.run(dgrtm.SOURCE_FIELD, every, with_source=True)
            errs.append(rel(sh.get_state(dgrtm.SOURCE_FIELD).cpu().numpy(), states[i]))
        tr = sh.forward()
        sh.adjoint(torch.from_numpy(data).cuda(), dgrtm.IMAGE_CHARACTERISTIC, (0.0, 0.0, 1.0), 0)
        e_img = rel(sh.image().cpu().numpy(), img_ref)
        e_tr = rel(tr.cpu().numpy(), tr_ref)
        _say(f"{name}: source field after " + ", ".join(f"{(i + 1) * every * 4} local steps {e:.2e}"
                                                       for i, e in enumerate(errs)) +
             f"; traces {e_tr:.2e}; image {e_img:.2e}")
        tol = 1e-5 if prec == dgrtm.FP32 else 1e-4
        assert max(errs) < tol and e_tr < tol and e_img < 1e-4
        del sh

