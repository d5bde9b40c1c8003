"""FP64 mesh connectivity and geometric factors for the DG oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the nodal-DG section (mesh of tetrahedra, Lagrange nodes mapped from
the reference element) and the appendix (affine map Psi_k, its Jacobian J_k,
the face Jacobians J_{k,f}).  The geometric factors used in the right-hand
side are the entries of the INVERSE Jacobian dr_j/dx_i (the chain rule needs
these; the paper's formula writes dPsi_i/dr_j).

Face-to-face node matching is done geometrically (nearest node), the plain
textbook way; the GPU library matches face nodes combinatorially instead, so
the two must agree exactly on the integer maps.
"""
from __future__ import annotations

import numpy as np

from .refelem import FACE_VERTS, RefElement

BC_INTERIOR, BC_RIGID, BC_TRANSPARENT, BC_FREE = 0, 1, 2, 3


def orient(verts: np.ndarray, etov: np.ndarray) -> np.ndarray:
    """Swap local vertices 2 and 3 where the signed volume is negative."""
    v = verts[etov]
    det = np.einsum("ij,ij->i", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))
    if np.any(det == 0):
        raise ValueError("degenerate element")
    out = etov.copy()
    neg = det < 0
    out[neg, 2], out[neg, 3] = etov[neg, 3], etov[neg, 2]
    return out


class OMesh:
    """Connectivity, node coordinates and geometry of a tetrahedral mesh (user element order)."""

    def __init__(self, ref: RefElement, verts: np.ndarray, etov: np.ndarray, bc_default: int = BC_RIGID,
                 face_bc: np.ndarray | None = None):
        self.ref = ref
        self.verts = np.asarray(verts, dtype=np.float64)
        self.etov = orient(self.verts, np.asarray(etov, dtype=np.int64))
        K = self.K = self.etov.shape[0]
        N, Np, Nfp = ref.N, ref.Np, ref.Nfp

        # --- face connectivity through sorted global vertex triples
        owners: dict[tuple, list] = {}
        for k in range(K):
            for f, lv in enumerate(FACE_VERTS):
                key = tuple(sorted(int(self.etov[k, i]) for i in lv))
                owners.setdefault(key, []).append((k, f))
        self.EToE = np.tile(np.arange(K)[:, None], (1, 4))
        self.EToF = np.tile(np.arange(4)[None, :], (K, 1))
        for key, lst in owners.items():
            if len(lst) > 2:
                raise ValueError("non-manifold face")
            if len(lst) == 2:
                (k1, f1), (k2, f2) = lst
                self.EToE[k1, f1], self.EToF[k1, f1] = k2, f2
                self.EToE[k2, f2], self.EToF[k2, f2] = k1, f1
        self.is_bdry = self.EToE == np.arange(K)[:, None]
        self.bc = np.zeros((K, 4), dtype=np.int64)
        if face_bc is not None:
            self.bc[:] = np.asarray(face_bc)
        else:
            self.bc[:] = bc_default
        self.bc[~self.is_bdry] = BC_INTERIOR

        # --- affine map x = -(1+r+s+t)/2 v0 + (1+r)/2 v1 + (1+s)/2 v2 + (1+t)/2 v3
        v = self.verts[self.etov]                       # (K,4,3)
        r, s, t = ref.rst[:, 0], ref.rst[:, 1], ref.rst[:, 2]
        self.x = (np.einsum("n,kd->knd", -(1 + r + s + t) / 2, v[:, 0]) +
                  np.einsum("n,kd->knd", (1 + r) / 2, v[:, 1]) +
                  np.einsum("n,kd->knd", (1 + s) / 2, v[:, 2]) +
                  np.einsum("n,kd->knd", (1 + t) / 2, v[:, 3]))   # (K,Np,3)
        A = np.stack([(v[:, 1] - v[:, 0]) / 2, (v[:, 2] - v[:, 0]) / 2, (v[:, 3] - v[:, 0]) / 2], axis=2)
        self.J = np.linalg.det(A)                        # dx/dr columns -> det
        if np.any(self.J <= 0):
            raise ValueError("non-positive Jacobian")
        Ainv = np.linalg.inv(A)                          # rows: grad r, grad s, grad t
        self.grad = Ainv                                 # (K, 3 [r,s,t], 3 [x,y,z])
        # outward face normals from the inverse-metric rows
        nraw = np.stack([-Ainv[:, 2], -Ainv[:, 1], Ainv[:, 0] + Ainv[:, 1] + Ainv[:, 2], -Ainv[:, 0]], axis=1)
        self.Fscale = np.linalg.norm(nraw, axis=2)      # (K,4) = J_f / J
        self.n = nraw / self.Fscale[:, :, None]         # (K,4,3)
        self.sJ = self.Fscale * self.J[:, None]

        # --- face node matching: for (k,f,i) the index i' on the neighbour face
        Fm = ref.Fmask                                   # (4,Nfp)
        self.nbr_node = np.tile(np.arange(Nfp)[None, None, :], (K, 4, 1))
        kk, ff = np.nonzero(~self.is_bdry)
        for lo in range(0, kk.size, 20000):
            k1, f1 = kk[lo:lo + 20000], ff[lo:lo + 20000]
            k2, f2 = self.EToE[k1, f1], self.EToF[k1, f1]
            xa = self.x[k1[:, None], Fm[f1]]               # (n,Nfp,3)
            xb = self.x[k2[:, None], Fm[f2]]
            d = np.linalg.norm(xa[:, :, None, :] - xb[:, None, :, :], axis=3)
            m = d.argmin(axis=2)
            dmin = np.take_along_axis(d, m[:, :, None], axis=2)[:, :, 0]
            scale = np.linalg.norm(xa.max(1) - xa.min(1), axis=1)
            if np.any(dmin > 1e-9 * scale[:, None]):
                raise ValueError("face nodes do not match")
            if np.any(np.sort(m, axis=1) != np.arange(Nfp)[None, :]):
                raise ValueError("face node matching is not a permutation")
            self.nbr_node[k1, f1] = m
        # volume-node maps in the paper's vmapM/vmapP sense (global node id k*Np+n)
        self.vmapM = (np.arange(K)[:, None, None] * Np + Fm[None, :, :])
        k2 = self.EToE[:, :, None]
        f2 = self.EToF[:, :, None]
        self.vmapP = k2 * Np + Fm[f2, self.nbr_node]
        self.vmapP = np.where(self.is_bdry[:, :, None], self.vmapM, self.vmapP)

    @property
    def volume(self) -> np.ndarray:
        return self.J * (4.0 / 3.0)


def face_areas(verts: np.ndarray, etov: np.ndarray) -> np.ndarray:
    """(K,4) face areas, each as half the norm of an edge cross product."""
    v = verts[etov]
    out = np.zeros((etov.shape[0], 4))
    for f, (a, b, c) in enumerate(FACE_VERTS):
        e1 = v[:, b] - v[:, a]
        e2 = v[:, c] - v[:, a]
        cr = np.cross(e1, e2)
        out[:, f] = 0.5 * np.sqrt(cr[:, 0] * cr[:, 0] + cr[:, 1] * cr[:, 1] + cr[:, 2] * cr[:, 2])
    return out


def local_dt(verts: np.ndarray, etov: np.ndarray, c: np.ndarray, N: int, cfl: float = 0.15) -> np.ndarray:
    """Largest local time step dt_k = cfl * l_k / ((N+1)^2 c_k) of every element.

    l_k is the smallest distance between a face and its opposite vertex, i.e.
    3*V_k / max_f A_f (single-rate time-step formula of the validation section,
    reused as the local CFL condition).  Written as explicit element-wise FP64
    operations in a fixed order so that level assignment is reproducible.
    """
    v = verts[etov]
    e1 = v[:, 1] - v[:, 0]
    e2 = v[:, 2] - v[:, 0]
    e3 = v[:, 3] - v[:, 0]
    cx = e2[:, 1] * e3[:, 2] - e2[:, 2] * e3[:, 1]
    cy = e2[:, 2] * e3[:, 0] - e2[:, 0] * e3[:, 2]
    cz = e2[:, 0] * e3[:, 1] - e2[:, 1] * e3[:, 0]
    vol = np.abs(e1[:, 0] * cx + e1[:, 1] * cy + e1[:, 2] * cz) / 6.0
    amax = np.zeros(etov.shape[0])
    for (a, b, cc) in FACE_VERTS:
        f1 = v[:, b] - v[:, a]
        f2 = v[:, cc] - v[:, a]
        gx = f1[:, 1] * f2[:, 2] - f1[:, 2] * f2[:, 1]
        gy = f1[:, 2] * f2[:, 0] - f1[:, 0] * f2[:, 2]
        gz = f1[:, 0] * f2[:, 1] - f1[:, 1] * f2[:, 0]
        area = 0.5 * np.sqrt(gx * gx + gy * gy + gz * gz)
        amax = np.maximum(amax, area)
    ell = 3.0 * vol / amax
    return cfl * ell / (float((N + 1) * (N + 1)) * c)


def lts_levels(dt: np.ndarray, EToE: np.ndarray, n_levels_max: int):
    """Multi-rate level of every element (1 = coarsest), following the time-stepping section.

    dt_local = min_k dt_k; level l_k is the smallest l in [1, L] with
    2^(L-l) dt_local <= dt_k (elements needing more doublings stay at level 1);
    then levels are raised until face neighbours differ by at most one
    (fixed point of l_k <- max(l_k, max_nbr l - 1)); finally empty coarse levels
    are removed (L shrinks, dt_local is unchanged).
    Returns (levels int64 (K,), L, dt_local).
    """
    L = int(n_levels_max)
    dt_local = float(dt.min())
    lev = np.full(dt.shape[0], L, dtype=np.int64)
    for l in range(L, 0, -1):
        ok = (2.0 ** (L - l)) * dt_local <= dt
        lev = np.where(ok, l, lev)
    while True:
        nb = lev[EToE].max(axis=1)
        new = np.maximum(lev, nb - 1)
        if np.array_equal(new, lev):
            break
        lev = new
    while L > 1 and not np.any(lev == 1):
        lev = lev - 1
        L -= 1
    return lev, L, dt_local
