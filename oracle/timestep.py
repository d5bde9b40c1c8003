"""FP64 time integrators for the DG oracle: LSERK(5,4), AB3 and multi-rate AB3.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Adams-Bashforth coefficients are derived, not typed in: A_s(theta) is the
  integral from 0 to theta of the Lagrange polynomial l_s on the time nodes
  {0, -1, -2} (time-stepping section, eq. updateAB and updateABcoarse; the
  imaging section, eq. ABrepS/ABrepR).  a_s = A_s(1), b_s = A_s(1/2); the
  tests pin these against the values the paper prints.
* The multi-rate scheme follows the forward time-stepping procedure (Alg. 1):
  per local step, the rhs of every element whose unknowns live at t_start;
  then, from the finest to the coarsest level, the AB3 update of the levels
  due at t_new (q and the trace copies qf); then the half-step traces of the
  coarse neighbours of elements evaluated at t_new (b_s coefficients; the
  paper's "b_f" is read as b_s).
* LSERK(5,4): the 5-stage 4th-order 2N-storage Runge-Kutta scheme of
  Carpenter and Kennedy (1994), used for the single-rate low-storage eigenmode
  run (not a scheme of the paper).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from .dg import Operator

NODES = (0, -1, -2)


def _lagrange_poly(s: int) -> list[Fraction]:
    """Coefficients (ascending powers) of the Lagrange polynomial l_s on NODES (s = 0,1,2)."""
    coef = [Fraction(1)]
    for j, xj in enumerate(NODES):
        if j == s:
            continue
        den = Fraction(NODES[s] - xj)
        new = [Fraction(0)] * (len(coef) + 1)
        for i, a in enumerate(coef):
            new[i + 1] += a / den
            new[i] += -xj * a / den
        coef = new
    return coef


def A_poly(s: int) -> list[Fraction]:
    """Coefficients of A_s(theta) = int_0^theta l_s."""
    l = _lagrange_poly(s)
    return [Fraction(0)] + [a / (i + 1) for i, a in enumerate(l)]


def poly_eval(c, x):
    return sum(a * x ** i for i, a in enumerate(c))


def poly_mul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def poly_int01(c):
    return sum(a / (i + 1) for i, a in enumerate(c))


def poly_reflect(c):
    """Coefficients of p(1 - theta)."""
    out = [Fraction(0)] * len(c)
    for i, a in enumerate(c):
        # (1 - x)^i
        for j in range(i + 1):
            from math import comb
            out[j] += a * comb(i, j) * (-1) ** j
    return out


def ab_coefficients():
    """Exact rationals: a (full step), b (half step), ebar, C (same direction), Cmix (opposite)."""
    A = [A_poly(s) for s in range(3)]
    a = [poly_eval(A[s], Fraction(1)) for s in range(3)]
    b = [poly_eval(A[s], Fraction(1, 2)) for s in range(3)]
    ebar = [poly_int01(A[s]) for s in range(3)]
    C = [[poly_int01(poly_mul(A[i], A[j])) for j in range(3)] for i in range(3)]
    Cmix = [[poly_int01(poly_mul(A[i], poly_reflect(A[j]))) for j in range(3)] for i in range(3)]
    return a, b, ebar, C, Cmix


_A, _B, _E, _C, _CM = ab_coefficients()
AB_A = np.array([float(x) for x in _A])
AB_B = np.array([float(x) for x in _B])


def lserk4_coefficients():
    """Carpenter-Kennedy (1994) 5-stage 4th-order 2N-storage coefficients (a, b, c)."""
    a = np.array([0.0,
                  -567301805773.0 / 1357537059087.0,
                  -2404267990393.0 / 2016746695238.0,
                  -3550918686646.0 / 2091501179385.0,
                  -1275806237668.0 / 842570457699.0])
    b = np.array([1432997174477.0 / 9575080441755.0,
                  5161836677717.0 / 13612068292357.0,
                  1720146321549.0 / 2090206949498.0,
                  3134564353537.0 / 4481467310338.0,
                  2277821191437.0 / 14882151754819.0])
    c = np.array([0.0,
                  1432997174477.0 / 9575080441755.0,
                  2526269341429.0 / 6820363183890.0,
                  2006345519317.0 / 3224310063776.0,
                  2802321613138.0 / 2924317926251.0])
    return a, b, c


def lserk4(op: Operator, q: np.ndarray, dt: float, nsteps: int, t0: float = 0.0, src=None) -> np.ndarray:
    a, b, c = lserk4_coefficients()
    q = q.copy()
    res = np.zeros_like(q)
    t = t0
    for _ in range(nsteps):
        for i in range(5):
            r = op.rhs(q)
            if src is not None:
                src(r, t + c[i] * dt)
            res = a[i] * res + dt * r
            q = q + b[i] * res
        t += dt
    return q


def ab3(op: Operator, q: np.ndarray, dt: float, nsteps: int, hist=None, t0: float = 0.0, src=None,
        reversed_time: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """Single-rate AB3.  hist: (2,K,4,Np) rhs at the two previous steps (newest first), or zeros."""
    q = q.copy()
    h = np.zeros((2,) + q.shape) if hist is None else np.array(hist, dtype=np.float64)
    for n in range(nsteps):
        t = t0 + n * dt
        r = op.rhs_reversed(q) if reversed_time else op.rhs(q)
        if src is not None:
            src(r, t)
        q = q + dt * (AB_A[0] * r + AB_A[1] * h[0] + AB_A[2] * h[1])
        h = np.stack([r, h[0]])
    return q, h


class MRAB:
    """Multi-rate AB3 of the forward time-stepping procedure (Alg. 1), FP64.

    levels: (K,) in 1..L, 1 = coarsest; Delta t_l = 2^(L-l) dt_local; one global step is
    2^(L-1) local steps.  `reversed_time` integrates dq/ds = -L(q; -tau) (backward run).
    `src(r, t_start, elems)` may add source terms into r (rows for `elems`).
    `on_eval(k_idx, step_idx, q_k, hist_k)` observes each element-step before its update (for
    imaging); `on_update(k_idx, step_idx)` is called after the update of the elements `k_idx`,
    step_idx being their new own step.  `replay(elems, n)` returns, for a boundary-trace replay
    run, the exterior traces (len(elems), 4, Nfp, 2) of the elements evaluated at local step n.
    """

    def __init__(self, op: Operator, levels: np.ndarray, L: int, dt_local: float,
                 reversed_time: bool = False, src=None, on_eval=None, on_update=None, replay=None):
        self.op = op
        self.lev = np.asarray(levels, dtype=np.int64)
        self.L = int(L)
        self.dt_local = float(dt_local)
        self.rev = reversed_time
        self.src = src
        self.on_eval = on_eval
        self.on_update = on_update
        self.replay = replay
        self.n = 0
        K = op.m.K
        self.q = np.zeros((K, 4, op.ref.Np))
        self.hist = np.zeros((K, 3, 4, op.ref.Np))     # newest first
        self.qf = op.traces(self.q)
        self.stride = 2 ** (self.L - self.lev)          # local steps per own step

    def set_state(self, q, hist2=None):
        """State at the start and, optionally, the AB3 history hist2 = (r(-dt), r(-2 dt)) of every
        element at its own step (the first update then uses r(0), r(-dt), r(-2 dt), eq. updateAB)."""
        self.q = np.array(q, dtype=np.float64)
        self.qf = self.op.traces(self.q)
        self.hist[:] = 0.0
        if hist2 is not None:
            # local_step shifts the history one slot before it stores the new rhs in slot 0
            self.hist[:, 0] = hist2[0]
            self.hist[:, 1] = hist2[1]

    @property
    def n_local(self) -> int:
        return 2 ** (self.L - 1)

    def local_step(self):
        op = self.op
        n = self.n
        dtl = self.dt_local * self.stride                # (K,) own step
        t_start = n * self.dt_local
        ev = np.nonzero(n % self.stride == 0)[0]          # unknowns evaluated at t_start
        rp = None if self.replay is None else self.replay(ev, n)
        r = (op.rhs_reversed(self.q, self.qf, elems=ev, replay=rp) if self.rev
             else op.rhs(self.q, self.qf, elems=ev, replay=rp))
        if self.src is not None:
            self.src(r, t_start, ev)
        self.hist[ev, 2] = self.hist[ev, 1]
        self.hist[ev, 1] = self.hist[ev, 0]
        self.hist[ev, 0] = r
        if self.on_eval is not None:
            self.on_eval(ev, n // self.stride[ev], self.q[ev], self.hist[ev])
        due = (n + 1) % self.stride == 0                  # evaluated at t_new
        for l in range(self.L, 0, -1):
            ks = np.nonzero(due & (self.lev == l))[0]
            if ks.size == 0:
                continue
            h = self.hist[ks]
            step = dtl[ks][:, None, None]
            self.q[ks] = self.q[ks] + step * (AB_A[0] * h[:, 0] + AB_A[1] * h[:, 1] + AB_A[2] * h[:, 2])
            self.qf[ks] = op.traces(self.q, ks)
            if self.on_update is not None:
                self.on_update(ks, (n + 1) // self.stride[ks])
        # coarse neighbours of elements evaluated at t_new get half-step traces
        nb = op.m.EToE
        touched = np.zeros(op.m.K, dtype=bool)
        dk = np.nonzero(due)[0]
        touched[nb[dk].ravel()] = True
        cn = np.nonzero(touched & ~due)[0]
        if cn.size:
            # they must sit exactly at the middle of their own step
            assert np.all((n + 1) % self.stride[cn] == self.stride[cn] // 2)
            h = self.hist[cn]
            step = dtl[cn][:, None, None]
            qh = self.q[cn] + step * (AB_B[0] * h[:, 0] + AB_B[1] * h[:, 1] + AB_B[2] * h[:, 2])
            self.qf[cn] = op.traces_of(qh, cn)
        self.n += 1

    def global_step(self):
        for _ in range(self.n_local):
            self.local_step()
