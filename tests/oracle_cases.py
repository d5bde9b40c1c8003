"""Small oracle set-ups shared by the CPU pin tests and the GPU parity tests (oracle side only)."""
from functools import lru_cache

import numpy as np

from oracle.dg import Operator
from oracle.mesh import BC_RIGID, BC_TRANSPARENT, OMesh, local_dt, lts_levels
from oracle.refelem import FACE_VERTS, get_ref
from paper_1506_00907_amd import inputs as I


@lru_cache(maxsize=None)
def case(name: str, bc: int = BC_TRANSPARENT, n_levels: int = 3):
    m, rho, c, N = I.config_mesh(name)
    ref = get_ref(N)
    M = OMesh(ref, m.verts, m.etov, bc_default=bc)
    op = Operator(M, rho, c)
    dt = local_dt(M.verts, M.etov, c, N)
    lev, L, dtl = lts_levels(dt, M.EToE, n_levels)
    return m, op, lev, L, dtl


def eigenmode(M, t):
    """Rigid unit-box eigenmode (rho = c = 1): p = cos(pi x)cos(pi y)cos(pi z)cos(w t), w = pi sqrt(3)."""
    w = np.pi * np.sqrt(3.0)
    x, y, z = M.x[..., 0], M.x[..., 1], M.x[..., 2]
    pi = np.pi
    q = np.zeros((M.K, 4, M.ref.Np))
    q[:, 0] = np.cos(pi * x) * np.cos(pi * y) * np.cos(pi * z) * np.cos(w * t)
    q[:, 1] = pi / w * np.sin(pi * x) * np.cos(pi * y) * np.cos(pi * z) * np.sin(w * t)
    q[:, 2] = pi / w * np.cos(pi * x) * np.sin(pi * y) * np.cos(pi * z) * np.sin(w * t)
    q[:, 3] = pi / w * np.cos(pi * x) * np.cos(pi * y) * np.sin(pi * z) * np.sin(w * t)
    return q


def oracle_shot(op, lev, L, dtl, n_global, spec):
    """The oracle's RTM shot for a shot spec (source point, Ricker wavelet, receivers)."""
    from oracle import source as OS
    from oracle.rtm import Shot as OShot
    M = op.m
    se = OS.locate(M, spec.src[None])[0]
    sw = OS.delta_weights(M, np.array([se]), spec.src[None])[0]
    re = OS.locate(M, spec.rec)
    return OShot(op, lev, L, dtl, n_global, se, sw, lambda t: OS.ricker(t, spec.f_peak, spec.t_peak), re,
                 OS.interp_rows(M, re, spec.rec), OS.delta_weights(M, re, spec.rec))


def neighbourhood_operator(N, verts, etov, rho, c, elems, bc_default=BC_TRANSPARENT, face_bc=None):
    """The oracle's operator on the sub-mesh made of `elems` and their face neighbours (elements
    sharing a sorted vertex triple with one of them).  An element's rhs needs only its own state
    and its neighbours' traces, so on this sub-mesh the oracle gives the whole mesh's rhs at `elems`
    without setting up the whole mesh.  Returns (operator, sub-mesh elements, positions of `elems`
    in the sub-mesh)."""
    verts = np.asarray(verts, dtype=np.float64)
    et = np.asarray(etov, dtype=np.int64)
    elems = np.asarray(elems, dtype=np.int64)
    nv = np.int64(verts.shape[0])
    f = np.sort(et[:, np.array(FACE_VERTS)], axis=2)
    key = (f[..., 0] * nv + f[..., 1]) * nv + f[..., 2]
    sub = np.flatnonzero(np.isin(key, key[elems].ravel()).any(axis=1))
    used = np.unique(et[sub])
    remap = np.full(verts.shape[0], -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    fb = None if face_bc is None else np.asarray(face_bc)[sub]
    om = OMesh(get_ref(N), verts[used], remap[et[sub]], bc_default=bc_default, face_bc=fb)
    op = Operator(om, np.asarray(rho, dtype=np.float64)[sub], np.asarray(c, dtype=np.float64)[sub])
    return op, sub, np.searchsorted(sub, elems)
