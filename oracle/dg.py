"""FP64 semi-discrete DG operator for the acoustic pressure-velocity system.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the model section (the p-v system and its boundary conditions) and
the nodal-DG section with its appendix (the strong-form element equations
with penalty fluxes):

  dp_k/dt   = - rho c^2 sum_j D_j U_j          - sum_f Fscale_f LIFT_f P^p_f
  dv_ik/dt  = - (1/rho) sum_j g_ji (D_j p)     - sum_f Fscale_f LIFT_f P^{v_i}_f

with U_j = sum_i g_ji v_i, g_ji = dr_j/dx_i (inverse Jacobian), and penalties

  P^p     = 1/2 rho c^2 ( n.[[v]] - tau_p [[p]] )
  P^{v_i} = 1/2 n_i/rho ( [[p]] - tau_v n.[[v]] ),    [[a]] = a+ - a-.

Readings where the paper is silent or inconsistent:
  * the 1/2 of the weak form is kept (the appendix drops it);
  * at a face between two media tau is the same on both sides:
    tau_p = 2/(Z- + Z+), tau_v = (Z- + Z+)/2 with Z = rho c (equal to the
    paper's upwind values in a homogeneous medium);
  * exterior states at the domain boundary: rigid wall p+ = p-,
    v+ = v- - 2(n.v-)n; free surface p+ = -p-, v+ = v-; transparent q+ = 0;
    on boundary faces tau_p = 1/Z-, tau_v = Z-;
  * backward-in-time runs use tau -> -tau (strictly negative penalties);
  * boundary-trace replay (the source field re-simulated backward in time, RTM
    procedure of the model section): on every boundary face the exterior state
    is the trace the forward run had there at the same time, p+ = p-_fwd and
    n.v+ = (n.v-)_fwd, whatever the boundary type; tau keeps its boundary value
    (the face-symmetric value with equal impedances on both sides).
"""
from __future__ import annotations

import numpy as np

from .mesh import BC_FREE, BC_RIGID, BC_TRANSPARENT, OMesh


class Operator:
    """The DG right-hand side of one mesh + material model."""

    def __init__(self, mesh: OMesh, rho: np.ndarray, c: np.ndarray):
        self.m = mesh
        self.ref = mesh.ref
        self.rho = np.asarray(rho, dtype=np.float64)
        self.c = np.asarray(c, dtype=np.float64)
        Z = self.rho * self.c
        Zp = Z[mesh.EToE]                              # neighbour impedance (self on boundary)
        Zm = Z[:, None]
        self.tau_p = np.where(mesh.is_bdry, 1.0 / Zm, 2.0 / (Zm + Zp))
        self.tau_v = np.where(mesh.is_bdry, Zm, 0.5 * (Zm + Zp))

    # ------------------------------------------------------------------ traces
    def traces(self, q: np.ndarray, elems=None) -> np.ndarray:
        """(K,4,Nfp,2): p and n.v (own outward normal) at each face node (rows `elems` if given)."""
        Fm = self.ref.Fmask
        if elems is not None:
            q = q[elems]
        nrm = self.m.n if elems is None else self.m.n[elems]
        p = q[:, 0][:, Fm]                              # (K,4,Nfp)
        v = q[:, 1:4][:, :, Fm]                         # (K,3,4,Nfp)
        nv = np.einsum("kfd,kdfi->kfi", nrm, v)
        return np.stack([p, nv], axis=3)

    def traces_of(self, qk: np.ndarray, elems) -> np.ndarray:
        """Traces of the element states qk (n,4,Np) belonging to elements `elems`."""
        Fm = self.ref.Fmask
        nrm = self.m.n[elems]
        p = qk[:, 0][:, Fm]
        v = qk[:, 1:4][:, :, Fm]
        return np.stack([p, np.einsum("kfd,kdfi->kfi", nrm, v)], axis=3)

    # ------------------------------------------------------------------ rhs
    def rhs(self, q: np.ndarray, qf: np.ndarray | None = None, tau_sign: float = 1.0,
            elems: np.ndarray | None = None, replay: np.ndarray | None = None) -> np.ndarray:
        """Right-hand side of the elements `elems` (all if None).

        q: (K,4,Np) nodal fields (p, vx, vy, vz).  qf: (K,4,Nfp,2) trace copies
        used for the surface terms (both sides), as in the surface kernel of the
        paper; if None the traces of q are used.  replay: (n,4,Nfp,2) recorded
        traces (p, n.v with the element's own normal) of the rows `elems`; where
        given, they are the exterior state on every boundary face.
        """
        m, R = self.m, self.ref
        if qf is None:
            qf = self.traces(q)
        ks = np.arange(m.K) if elems is None else np.asarray(elems)
        rho, c = self.rho[ks], self.c[ks]
        rc2 = rho * c * c
        G = m.grad[ks]                                  # (n,3,3) [j=r,s,t][i=x,y,z]
        p = q[ks, 0]
        v = q[ks, 1:4]                                  # (n,3,Np)
        # volume terms
        U = np.einsum("kji,kin->kjn", G, v)             # U_j = sum_i dr_j/dx_i v_i
        D = (R.Dr, R.Ds, R.Dt)
        divv = sum(U[:, j] @ D[j].T for j in range(3))
        out = np.zeros((ks.size, 4, R.Np))
        out[:, 0] = -rc2[:, None] * divv
        Dp = np.stack([p @ D[j].T for j in range(3)], axis=1)  # (n,3,Np)
        gradp = np.einsum("kji,kjn->kin", G, Dp)
        out[:, 1:4] = -gradp / rho[:, None, None]

        # surface terms
        pM = qf[ks, :, :, 0]                            # (n,4,Nfp)
        nvM = qf[ks, :, :, 1]
        k2 = m.EToE[ks]
        f2 = m.EToF[ks]
        i2 = m.nbr_node[ks]
        pP = qf[k2[:, :, None], f2[:, :, None], i2, 0]
        nvP = -qf[k2[:, :, None], f2[:, :, None], i2, 1]   # n- . v+ = -(n+ . v+)
        bc = m.bc[ks][:, :, None]
        pP = np.where(bc == BC_RIGID, pM, pP)
        nvP = np.where(bc == BC_RIGID, -nvM, nvP)
        pP = np.where(bc == BC_FREE, -pM, pP)
        nvP = np.where(bc == BC_FREE, nvM, nvP)
        pP = np.where(bc == BC_TRANSPARENT, 0.0, pP)
        nvP = np.where(bc == BC_TRANSPARENT, 0.0, nvP)
        if replay is not None:
            bd = m.is_bdry[ks][:, :, None]
            pP = np.where(bd, replay[..., 0], pP)
            nvP = np.where(bd, replay[..., 1], nvP)
        dp = pP - pM
        dnv = nvP - nvM
        taup = tau_sign * self.tau_p[ks][:, :, None]
        tauv = tau_sign * self.tau_v[ks][:, :, None]
        Fs = m.Fscale[ks][:, :, None]
        Pp = 0.5 * rc2[:, None, None] * (dnv - taup * dp) * Fs      # (n,4,Nfp)
        Pv = 0.5 / rho[:, None, None] * (dp - tauv * dnv) * Fs      # scalar part of P^v
        Nfp = R.Nfp
        Lf = R.LIFT.reshape(R.Np, 4, Nfp)
        out[:, 0] -= Pp.reshape(ks.size, 4 * Nfp) @ R.LIFT.T
        g = np.stack([Pv[:, f] @ Lf[:, f].T for f in range(4)], axis=1)   # (n,4,Np)
        out[:, 1:4] -= np.einsum("kfd,kfn->kdn", m.n[ks], g)
        return out

    def rhs_reversed(self, q, qf=None, elems=None, replay=None):
        """Right-hand side in reversed time s = t_f - t: -L(q; -tau)."""
        return -self.rhs(q, qf, tau_sign=-1.0, elems=elems, replay=replay)

    # ------------------------------------------------------------------ energy
    def energy(self, q: np.ndarray) -> float:
        """1/2 sum_k integral(p^2/(rho c^2) + rho |v|^2)."""
        M = self.ref.M
        J = self.m.J
        e = 0.0
        e += np.einsum("k,kn,nm,km->", J / (self.rho * self.c ** 2), q[:, 0], M, q[:, 0])
        for d in range(1, 4):
            e += np.einsum("k,kn,nm,km->", J * self.rho, q[:, d], M, q[:, d])
        return 0.5 * e
