"""FP64 reverse-time migration with the characteristic imaging condition (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the model section (RTM procedure; classical condition eq. imageP and
characteristic condition eq. imageQ with q+- = p +- rho c e.v, e pointing up)
and the imaging section (exact time integral of the product of the two
fields' AB3 dense-output polynomials, computed right before each update).

The plain, non-checkpointed form: the source wavefield S is run forward from
rest and every element-step (q-_S at the step start and its rhs) is kept in
memory; the receiver wavefield R is run backward (reversed time, tau -> -tau)
from rest with the data injected at the receivers.  For each own-level step
[t_a, t_b] of an element, S is known by its dense output forward from t_a and
R by its dense output backward from t_b, so the per-step integral is

  dt q_S q_R + dt^2 sum_s ebar_s (q_S r~_R^(s) + r_S^(s) q_R)
             + dt^3 sum_{s1,s2} Cmix_{s1 s2} r_S^(s1) r~_R^(s2)

with ebar_s = int_0^1 A_s and Cmix = int_0^1 A_s1(th) A_s2(1-th) (derived
exactly in timestep.ab_coefficients).  The paper's printed formula is for two
fields both run backward; its dt^2 weights must read ebar_s, not a_s.
Independently, the same integral is evaluated by 8-point Gauss-Legendre
quadrature of the reconstructed polynomials (rtm(..., quadrature=True)).
"""
from __future__ import annotations

import numpy as np

from .dg import Operator
from .source import data_at
from .timestep import MRAB, A_poly, ab_coefficients, poly_eval

COND_PRESSURE, COND_CHARACTERISTIC = 0, 1


def _coeffs():
    a, b, e, C, Cm = ab_coefficients()
    return np.array([float(x) for x in e]), np.array([[float(x) for x in r] for r in Cm])


class Shot:
    """One RTM shot on the oracle: source (element, weights, wavelet samples) and receivers."""

    def __init__(self, op: Operator, levels, L, dt_local, n_global: int,
                 src_elem: int, src_w: np.ndarray, wavelet, rec_elem: np.ndarray, rec_l: np.ndarray,
                 rec_w: np.ndarray):
        self.op, self.lev, self.L, self.dt_local = op, np.asarray(levels), int(L), float(dt_local)
        self.n_global = int(n_global)
        self.n_local = 2 ** (self.L - 1)
        self.src_elem, self.src_w, self.wavelet = int(src_elem), src_w, wavelet
        self.rec_elem, self.rec_l, self.rec_w = rec_elem, rec_l, rec_w

    # ---------------------------------------------------------------- forward
    def forward(self, condition=COND_CHARACTERISTIC, up=(0.0, 0.0, 1.0), keep=True):
        """Run S; return traces (n_rec, n_global+1); keep per element-step q-_S and r-_S."""
        op = self.op
        K, Np = op.m.K, op.ref.Np
        up = np.asarray(up, dtype=np.float64)
        max_steps = self.n_global * self.n_local
        self.qS = np.zeros((max_steps, K, Np)) if keep else None
        self.rS = np.zeros((max_steps, K, Np)) if keep else None

        def src(r, t, ev):
            hit = np.nonzero(ev == self.src_elem)[0]
            if hit.size:
                r[hit[0], 0] += self.wavelet(t) * self.src_w

        def on_eval(ev, m, q, hist):
            if keep:
                self.qS[m, ev] = _split_rows(op, ev, q, up, -1.0, condition)
                self.rS[m, ev] = _split_rows(op, ev, hist[:, 0], up, -1.0, condition)

        st = MRAB(op, self.lev, self.L, self.dt_local, src=src, on_eval=on_eval)
        tr = np.zeros((self.rec_elem.size, self.n_global + 1))
        for g in range(self.n_global):
            st.global_step()
            tr[:, g + 1] = np.einsum("rn,rn->r", self.rec_l, st.q[self.rec_elem, 0])
        self.S_final = st.q.copy()
        return tr

    # ---------------------------------------------------------------- backward + image
    def adjoint(self, data: np.ndarray, condition=COND_CHARACTERISTIC, up=(0.0, 0.0, 1.0),
                g_image_start: int = 0, quadrature: bool = False):
        """Run R backward over [t_i, t_f] with the data injected; return the FP64 image (K, Np)."""
        op = self.op
        K, Np = op.m.K, op.ref.Np
        up = np.asarray(up, dtype=np.float64)
        ebar, Cm = _coeffs()
        img = np.zeros((K, Np))
        stride = 2 ** (self.L - self.lev)
        nl = self.n_local
        total = self.n_global * nl
        i_start = g_image_start * nl
        Aq = [A_poly(s) for s in range(3)]
        xg, wg = np.polynomial.legendre.leggauss(8)
        th = 0.5 * (xg + 1.0)
        wq = 0.5 * wg
        Ath = np.array([[float(poly_eval(Aq[s], t)) for t in th] for s in range(3)])        # A_s(th)
        Ath1 = np.array([[float(poly_eval(Aq[s], 1.0 - t)) for t in th] for s in range(3)])  # A_s(1-th)

        def src(r, s_t, ev):
            # physical time of this rhs: t = t_f - s  (in local steps: total - n)
            n = int(round(s_t / self.dt_local))
            d = data_at(data, nl, total - n)
            for j, k in enumerate(ev):
                hit = np.nonzero(self.rec_elem == k)[0]
                if hit.size:
                    r[j, 0] -= (d[hit][:, None] * self.rec_w[hit]).sum(0)

        def on_eval(ev, mR, q, hist):
            st_ = stride[ev]
            dt = self.dt_local * st_
            own = self.n_global * (nl // st_)              # own steps per run
            mS = own - mR - 1
            keep = mS * st_ >= i_start
            if not np.any(keep):
                return
            ev, mS, dt, q, hist = ev[keep], mS[keep], dt[keep], q[keep], hist[keep]
            qR = _split_rows(op, ev, q, up, +1.0, condition)
            rR = np.stack([_split_rows(op, ev, hist[:, s], up, +1.0, condition) for s in range(3)])
            qS = self.qS[mS, ev]
            rS = np.stack([np.where((mS - s >= 0)[:, None], self.rS[np.maximum(mS - s, 0), ev], 0.0)
                           for s in range(3)])
            d1 = dt[:, None]
            if not quadrature:
                inc = d1 * qS * qR
                for s in range(3):
                    inc += d1 ** 2 * ebar[s] * (qS * rR[s] + rS[s] * qR)
                for s1 in range(3):
                    for s2 in range(3):
                        inc += d1 ** 3 * Cm[s1, s2] * rS[s1] * rR[s2]
            else:
                inc = np.zeros_like(qS)
                for iq in range(th.size):
                    fS = qS + d1 * sum(Ath[s, iq] * rS[s] for s in range(3))
                    fR = qR + d1 * sum(Ath1[s, iq] * rR[s] for s in range(3))
                    inc += wq[iq] * d1 * fS * fR
            np.add.at(img, ev, inc)

        st = MRAB(op, self.lev, self.L, self.dt_local, reversed_time=True, src=src, on_eval=on_eval)
        for g in range(self.n_global - g_image_start):
            st.global_step()
        self.R_final = st.q.copy()
        return img


def _split_rows(op: Operator, ev, q, up, sign, condition):
    if condition == COND_PRESSURE:
        return q[:, 0].copy()
    Z = (op.rho[ev] * op.c[ev])[:, None]
    uv = up[0] * q[:, 1] + up[1] * q[:, 2] + up[2] * q[:, 3]
    return q[:, 0] + sign * Z * uv
