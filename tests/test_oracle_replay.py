"""Pins of the oracle's boundary-trace replay (the paper's own storage strategy: the source field
re-simulated backward in time from its final state with the boundary traces of the forward run)
and of the trapezoid variant of the image integral.

- The both-backward image formula (weights ebar_s and the printed matrix C) equals Gauss-Legendre
  quadrature of the product of the two fields' backward AB3 dense outputs.
- The replayed image converges at third order in the time step (imaging section), which fixes the
  pairing of the two backward runs, the time of every replayed trace and the start of the
  backward source run's AB3 history.
- Replaying the boundary traces brings a resolved pulse that has partly left the box back to its
  initial state, to an error that falls as the order N grows; without the replay (transparent
  boundaries in the backward run) or with the normal velocity of the replayed traces of the wrong
  sign, the part that left is lost.
- The trapezoid rule (eq. trapRule, sign read as "+") converges at second order where the
  integrand does not vanish at the ends of the image window, against third order for the exact
  integral of the same shot (the paper calls it first order).
"""
import numpy as np
import pytest

from oracle import source as S
from oracle.dg import Operator
from oracle.mesh import BC_TRANSPARENT, OMesh, local_dt, lts_levels
from oracle.refelem import get_ref
from oracle.rtm import COND_CHARACTERISTIC, COND_PRESSURE, Shot
from paper_1506_00907_amd import inputs as I
from tests.oracle_cases import case


def _order(a, b, c):
    return np.log2(np.linalg.norm(a - b) / np.linalg.norm(b - c))


def _tapered_shots(G0=30, n_ref=3):
    """The smooth shot of the third-order test of the checkpointed image (40 Hz Ricker peaking at
    1.5/f_p, data tapered to zero at t_f), at dt, dt/2, dt/4, with the boundary traces recorded."""
    m, op, lev, L, dtl = case("two_layer_small:4:4:3:2")
    M = op.m
    f_p = 40.0
    spec = I.rtm_shot(n_rec=4)
    se = S.locate(M, spec.src[None])[0]
    sw = S.delta_weights(M, np.array([se]), spec.src[None])[0]
    re = S.locate(M, spec.rec)
    out = []
    for r in range(n_ref):
        G = G0 * 2 ** r
        sh = Shot(op, lev, L, dtl / 2 ** r, G, se, sw, lambda t: S.ricker(t, f_p, 1.5 / f_p), re,
                  S.interp_rows(M, re, spec.rec), S.delta_weights(M, re, spec.rec))
        tr = sh.forward(record_boundary=True)
        tg = np.arange(G + 1) * (dtl / 2 ** r) * 2 ** (L - 1)
        half = tg[-1] / 2
        w = np.where(tg > half, (0.5 * (1.0 + np.cos(np.pi * (tg - half) / half))) ** 2, 1.0)
        out.append((sh, tr * w[None], G))
    return out


@pytest.fixture(scope="module")
def shots():
    return _tapered_shots()


@pytest.mark.parametrize("cond", [COND_CHARACTERISTIC, COND_PRESSURE])
def test_replay_formula_equals_quadrature(shots, cond):
    sh, data, G = shots[0]
    a = sh.adjoint_replay(data, condition=cond)
    b = sh.adjoint_replay(data, condition=cond, quadrature=True)
    assert np.abs(a).max() > 0
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def test_replay_image_converges_at_third_order(shots):
    full, back = [], []
    for sh, d, G in shots:
        full.append(sh.adjoint_replay(d))
        back.append(sh.S_back.copy())
    late = [sh.adjoint_replay(d, g_image_start=G // 2) for sh, d, G in shots]
    of, ol = _order(*full), _order(*late)
    # the re-simulated source field at t = 0 too: a first-order start of its AB3 history (zero
    # history: 1.7) or traces replayed one own step late (1.0) would show here
    ob = _order(*back)
    assert ob >= 2.5, ob
    assert np.abs(late[-1]).max() > 0.05 * np.abs(full[-1]).max()
    assert of >= 2.5, of
    assert ol >= 2.5, ol


def test_trapezoid_rule_is_second_order(shots):
    # The exact integral is third-order accurate, so the trapezoid rule's distance from it at the
    # same step is the trapezoid rule's own error.  The window starts at mid-run, where the
    # integrand does not vanish: the leading error term (dt^2/12 times the integrand's derivative
    # at the window ends) remains, and halving the step divides the error by about 4.  (Over the
    # whole run the integrand and its derivatives vanish at both ends and the error falls much
    # faster, as the Euler-Maclaurin formula says.)
    for replay in (False, True):
        errs = []
        for sh, d, G in shots[1:]:
            run = sh.adjoint_replay if replay else sh.adjoint
            trap = run(d, g_image_start=G // 2, rule="trapezoid")
            exact = run(d, g_image_start=G // 2)
            errs.append(np.linalg.norm(trap - exact) / np.linalg.norm(exact))
        order = np.log2(errs[0] / errs[1])
        assert 1.6 <= order <= 2.4, (replay, errs, order)
        assert errs[1] > 1e-4, (replay, errs)


def _pulse_shot(N):
    mm, rho, c, _ = I.config_mesh("two_layer_small:4:4:3:2")
    om = OMesh(get_ref(N), mm.verts, mm.etov, bc_default=BC_TRANSPARENT)
    op = Operator(om, rho, c)
    lev, L, dtl = lts_levels(local_dt(om.verts, om.etov, c, N), om.EToE, 3)
    x = om.x
    q0 = np.zeros((om.K, 4, om.ref.Np))
    q0[:, 0] = np.exp(-((x[..., 0] - 1.0) ** 2 + (x[..., 1] - 1.0) ** 2 + (x[..., 2] - 0.7) ** 2) / 0.3 ** 2)
    G = int(round(0.3 / (dtl * 2 ** (L - 1))))
    rec = np.array([[1.0, 1.0, 0.99]])
    re = S.locate(om, rec)
    sh = Shot(op, lev, L, dtl, G, 0, np.zeros(om.ref.Np), lambda t: 0.0, re, S.interp_rows(om, re, rec),
              S.delta_weights(om, re, rec))
    sh.forward(record_boundary=True, q0=q0)
    return sh, q0, G


def test_replay_brings_a_resolved_pulse_back():
    errs = []
    for N in (2, 3):
        sh, q0, G = _pulse_shot(N)
        # part of the pulse has left through the transparent boundary by t_f
        assert np.linalg.norm(sh.S_final) < 0.9 * np.linalg.norm(q0)
        sh.adjoint_replay(np.zeros((1, G + 1)))
        errs.append(np.linalg.norm(sh.S_back - q0) / np.linalg.norm(q0))
    assert errs[1] < 0.7 * errs[0], errs

    # planted mistakes (in the oracle, here on the CPU): no replay, and n.v replayed with the
    # wrong sign, both lose what left the box
    class NoReplay(Shot):
        def _replay_rows(self, ev, j):
            return np.zeros((ev.size, 4, self.op.ref.Nfp, 2))

    class Flipped(Shot):
        def _replay_rows(self, ev, j):
            o = super()._replay_rows(ev, j)
            o[..., 1] *= -1.0
            return o

    for cls in (NoReplay, Flipped):
        sh.__class__ = cls
        sh.adjoint_replay(np.zeros((1, G + 1)))
        bad = np.linalg.norm(sh.S_back - q0) / np.linalg.norm(q0)
        assert bad > 3 * errs[1], (cls.__name__, bad, errs[1])
