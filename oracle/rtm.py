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

The trapezoid rule of the imaging section (eq. trapRule, its sign read as "+")
is the variant rule="trapezoid": dt/2 (S R at the step start + S R at the step
end), taken from the fields' states at both ends of every own step.

The paper's own storage strategy (RTM procedure of the model section, the
backward-in-time paragraph of the time-stepping section and the section on
memory transfers) is Shot.forward(record_boundary=True) followed by
Shot.adjoint_replay: the forward run saves p and n.v at the boundary face nodes
after every own step of every element that has a boundary face, and the final
state; S is then re-simulated backward in time (tau -> -tau, the source with
sign -1) with the saved traces as the exterior state of every boundary face,
step by step together with R, and the image takes the both-backward form of
eq. updateABcorr: weights ebar_s in the dt^2 terms and the printed matrix C.
Where the paper is silent (how the backward source run starts its AB3
history), the history at t_f is extrapolated: the reversed-time rhs is
evaluated at the last three global times t_f, t_f - dt_g, t_f - 2 dt_g from
the forward states saved there (with the replayed boundary traces and the
source), and the quadratic through them is evaluated at t_f + dt_l and
t_f + 2 dt_l for every level (third-order accurate, like AB3 itself).
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
    def forward(self, condition=COND_CHARACTERISTIC, up=(0.0, 0.0, 1.0), keep=True, record_boundary=False,
                q0=None, snap_every=0, progress=None):
        """Run S; return traces (n_rec, n_global+1); keep per element-step q-_S and r-_S.

        q0: state at t = 0 (zero AB3 history); default: at rest.
        snap_every: also keep the state after every snap_every global steps (self.snaps).
        progress(g): called after every global step (long runs report their steps).

        record_boundary: also save the boundary traces after every own step of the elements that
        have a boundary face (self.bnd_rec: (n_bnd, J+1, 4, Nfp, 2), row j = own step j, row 0 the
        state at rest) and the states at the last three global times (self.q_end)."""
        op = self.op
        K, Np = op.m.K, op.ref.Np
        up = np.asarray(up, dtype=np.float64)
        max_steps = self.n_global * self.n_local
        self.qS = np.zeros((max_steps, K, Np)) if keep else None
        self.rS = np.zeros((max_steps, K, Np)) if keep else None
        on_update = None
        if record_boundary:
            bel = np.flatnonzero(op.m.is_bdry.any(axis=1))
            self.bnd_pos = np.full(K, -1, dtype=np.int64)
            self.bnd_pos[bel] = np.arange(bel.size)
            self.bnd_rec = np.zeros((bel.size, max_steps + 1, 4, op.ref.Nfp, 2))

            def on_update(ks, j):
                b = self.bnd_pos[ks]
                sel = b >= 0
                if np.any(sel):
                    self.bnd_rec[b[sel], j[sel]] = op.traces(st.q, ks[sel])
            self.q_end = {}

        def src(r, t, ev):
            hit = np.nonzero(ev == self.src_elem)[0]
            if hit.size:
                r[hit[0], 0] += self.wavelet(t) * self.src_w

        def on_eval(ev, m, q, hist):
            if keep:
                self.qS[m, ev] = _split_rows(op, ev, q, up, -1.0, condition)
                self.rS[m, ev] = _split_rows(op, ev, hist[:, 0], up, -1.0, condition)

        st = MRAB(op, self.lev, self.L, self.dt_local, src=src, on_eval=on_eval, on_update=on_update)
        if q0 is not None:
            st.set_state(q0)
        if record_boundary:
            self.q_end[0] = st.q.copy()
            b = self.bnd_pos >= 0
            self.bnd_rec[:, 0] = op.traces(st.q, np.flatnonzero(b))
        tr = np.zeros((self.rec_elem.size, self.n_global + 1))
        tr[:, 0] = np.einsum("rn,rn->r", self.rec_l, st.q[self.rec_elem, 0])
        self.snaps = []
        for g in range(self.n_global):
            st.global_step()
            tr[:, g + 1] = np.einsum("rn,rn->r", self.rec_l, st.q[self.rec_elem, 0])
            if record_boundary and g + 1 >= self.n_global - 2:
                self.q_end[g + 1] = st.q.copy()
            if snap_every and (g + 1) % snap_every == 0:
                self.snaps.append(st.q.copy())
            if progress is not None:
                progress(g + 1)
        self.S_final = st.q.copy()
        return tr

    # ---------------------------------------------------------------- backward + image
    def adjoint(self, data: np.ndarray, condition=COND_CHARACTERISTIC, up=(0.0, 0.0, 1.0),
                g_image_start: int = 0, quadrature: bool = False, rule: str = "exact", progress=None):
        """Run R backward over [t_i, t_f] with the data injected; return the FP64 image (K, Np).

        rule "exact": the dense-output integral (quadrature=True: by Gauss-Legendre quadrature);
        rule "trapezoid": dt/2 (S R at both ends of every own step), from the fields' states."""
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

        if rule == "trapezoid":
            steps_run = (self.n_global - g_image_start) * nl
            qR_st = np.zeros((steps_run, K, Np))

        def on_eval(ev, mR, q, hist):
            if rule == "trapezoid":
                qR_st[mR, ev] = _split_rows(op, ev, q, up, +1.0, condition)
                return
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
            if progress is not None:
                progress(g + 1)
        self.R_final = st.q.copy()
        if rule == "trapezoid":
            # S at the end of its last step is the final state; R at the end of its last step is R_final
            allk = np.arange(K)
            S_end = _split_rows(op, allk, self.S_final, up, -1.0, condition)
            R_end = _split_rows(op, allk, self.R_final, up, +1.0, condition)
            for l in np.unique(self.lev):
                ks = np.flatnonzero(self.lev == l)
                st_ = int(stride[ks[0]])
                own = self.n_global * (nl // st_)
                nR = (self.n_global - g_image_start) * (nl // st_)
                dt = self.dt_local * st_
                for mR in range(nR):
                    mS = own - mR - 1                       # S step [t_a, t_b], R step from t_b to t_a
                    S_a = self.qS[mS, ks]
                    S_b = self.qS[mS + 1, ks] if mS + 1 < own else S_end[ks]
                    R_b = qR_st[mR, ks]
                    R_a = qR_st[mR + 1, ks] if mR + 1 < nR else R_end[ks]
                    img[ks] += 0.5 * dt * (S_a * R_a + S_b * R_b)
        return img

    # ---------------------------------------------------------------- boundary-trace replay
    def _replay_rows(self, ev, j):
        """Exterior traces for elements ev at their own steps j (zeros where no boundary face)."""
        op = self.op
        out = np.zeros((ev.size, 4, op.ref.Nfp, 2))
        b = self.bnd_pos[ev]
        sel = (b >= 0) & (j >= 0)
        if np.any(sel):
            out[sel] = self.bnd_rec[b[sel], j[sel]]
        return out

    def _source_at(self, t):
        return self.wavelet(t) if t >= 0.0 else 0.0

    def backward_start_history(self):
        """AB3 history (r~(-dt_l), r~(-2 dt_l)) of the source field's backward run, per element:
        the reversed-time rhs at the global times t_f, t_f - dt_g, t_f - 2 dt_g (forward states
        saved there, replayed boundary traces, source with sign -1; at rest before t = 0)
        extrapolated quadratically to t_f + dt_l and t_f + 2 dt_l."""
        op = self.op
        K = op.m.K
        NG, nl = self.n_global, self.n_local
        dtg = self.dt_local * nl
        allk = np.arange(K)
        per_level = 2 ** (self.lev - 1)                  # own steps per global step
        r = []
        for i in range(3):
            G = NG - i
            q = self.S_final if i == 0 else (self.q_end[G] if G >= 0 else np.zeros_like(self.S_final))
            rep = self._replay_rows(allk, G * per_level if G >= 0 else np.full(K, -1))
            ri = op.rhs_reversed(q, None, replay=rep)
            ri[self.src_elem, 0] -= self._source_at(G * dtg) * self.src_w
            r.append(ri)
        rho = 2.0 ** (1 - self.lev.astype(np.float64))   # dt_l / dt_g per element

        def lag(tau):
            return [(tau + 1) * (tau + 2) / 2, -tau * (tau + 2), tau * (tau + 1) / 2]

        h = []
        for k in (1, 2):
            w = lag(k * rho)
            h.append(sum(w[i][:, None, None] * r[i] for i in range(3)))
        return h

    def adjoint_replay(self, data: np.ndarray, condition=COND_CHARACTERISTIC, up=(0.0, 0.0, 1.0),
                       g_image_start: int = 0, quadrature: bool = False, rule: str = "exact"):
        """Both fields backward over [t_i, t_f]: S re-simulated from its final state with the
        recorded boundary traces, R from rest with the data; returns the FP64 image (K, Np).
        Needs forward(record_boundary=True).  Also keeps self.S_back (S at t_i)."""
        op = self.op
        K, Np = op.m.K, op.ref.Np
        up = np.asarray(up, dtype=np.float64)
        a, b, e, C, Cm = ab_coefficients()
        ebar = np.array([float(x) for x in e])
        Cs = np.array([[float(x) for x in row] for row in C])
        img = np.zeros((K, Np))
        stride = 2 ** (self.L - self.lev)
        nl = self.n_local
        total = self.n_global * nl
        Aq = [A_poly(s) for s in range(3)]
        xg, wg = np.polynomial.legendre.leggauss(8)
        th = 0.5 * (xg + 1.0)
        wq = 0.5 * wg
        Ath = np.array([[float(poly_eval(Aq[s], t)) for t in th] for s in range(3)])
        cur = {}

        def src_S(r, s_t, ev):
            n = int(round(s_t / self.dt_local))
            hit = np.nonzero(ev == self.src_elem)[0]
            if hit.size:
                r[hit[0], 0] -= self._source_at((total - n) * self.dt_local) * self.src_w

        def src_R(r, s_t, ev):
            n = int(round(s_t / self.dt_local))
            d = data_at(data, nl, total - n)
            for j, k in enumerate(ev):
                hit = np.nonzero(self.rec_elem == k)[0]
                if hit.size:
                    r[j, 0] -= (d[hit][:, None] * self.rec_w[hit]).sum(0)

        def replay_S(ev, n):
            # backward local step n is physical local step total - n; own step j of the element
            return self._replay_rows(ev, (total - n) // stride[ev])

        def eval_S(ev, m, q, hist):
            cur["S"] = (ev, _split_rows(op, ev, q, up, -1.0, condition),
                        np.stack([_split_rows(op, ev, hist[:, s], up, -1.0, condition) for s in range(3)]))

        steps_run = (self.n_global - g_image_start) * nl
        if rule == "trapezoid":
            qS_st = np.zeros((steps_run, K, Np))
            qR_st = np.zeros((steps_run, K, Np))

        def eval_R(ev, m, q, hist):
            evS, qS, rS = cur.pop("S")
            assert np.array_equal(evS, ev)
            qR = _split_rows(op, ev, q, up, +1.0, condition)
            if rule == "trapezoid":
                qS_st[m, ev] = qS
                qR_st[m, ev] = qR
                return
            rR = np.stack([_split_rows(op, ev, hist[:, s], up, +1.0, condition) for s in range(3)])
            d1 = (self.dt_local * stride[ev])[:, None]
            if not quadrature:
                inc = d1 * qS * qR
                for s in range(3):
                    inc += d1 ** 2 * ebar[s] * (qS * rR[s] + rS[s] * qR)
                for s1 in range(3):
                    for s2 in range(3):
                        inc += d1 ** 3 * Cs[s1, s2] * rS[s1] * rR[s2]
            else:
                inc = np.zeros_like(qS)
                for iq in range(th.size):
                    fS = qS + d1 * sum(Ath[s, iq] * rS[s] for s in range(3))
                    fR = qR + d1 * sum(Ath[s, iq] * rR[s] for s in range(3))
                    inc += wq[iq] * d1 * fS * fR
            np.add.at(img, ev, inc)

        S = MRAB(op, self.lev, self.L, self.dt_local, reversed_time=True, src=src_S, on_eval=eval_S,
                 replay=replay_S)
        S.set_state(self.S_final, hist2=self.backward_start_history())
        R = MRAB(op, self.lev, self.L, self.dt_local, reversed_time=True, src=src_R, on_eval=eval_R)
        for _ in range(steps_run):
            S.local_step()
            R.local_step()
        self.S_back = S.q.copy()
        self.R_final = R.q.copy()
        if rule == "trapezoid":
            allk = np.arange(K)
            S_end = _split_rows(op, allk, S.q, up, -1.0, condition)
            R_end = _split_rows(op, allk, R.q, up, +1.0, condition)
            for l in np.unique(self.lev):
                ks = np.flatnonzero(self.lev == l)
                st_ = int(stride[ks[0]])
                nR = (self.n_global - g_image_start) * (nl // st_)
                dt = self.dt_local * st_
                for m in range(nR):
                    S_b, R_b = qS_st[m, ks], qR_st[m, ks]
                    S_a = qS_st[m + 1, ks] if m + 1 < nR else S_end[ks]
                    R_a = qR_st[m + 1, ks] if m + 1 < nR else R_end[ks]
                    img[ks] += 0.5 * dt * (S_a * R_a + S_b * R_b)
        return img


def _split_rows(op: Operator, ev, q, up, sign, condition):
    if condition == COND_PRESSURE:
        return q[:, 0].copy()
    Z = (op.rho[ev] * op.c[ev])[:, None]
    uv = up[0] * q[:, 1] + up[1] * q[:, 2] + up[2] * q[:, 3]
    return q[:, 0] + sign * Z * uv
