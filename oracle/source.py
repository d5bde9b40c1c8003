"""FP64 point sources, receivers and wavelets for the DG oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Point source (nodal-DG section, eq. sourceTerm): the Dirac delta is replaced
  by its L2 projection on the element's polynomial space,
  delta~ = sum_n w_n l_n with M_k w = l(x0), i.e. w = M_k^{-1} l(x0).
  The source is added to the pressure equation as f(t) * w, following the PDE
  (no rho c^2 factor; the weak form as printed would add one).
* The element holding a point is the lowest-numbered element whose
  barycentric coordinates of the point are all >= -1e-12.
* Recording: the element polynomial evaluated at the receiver, p(x_r) = l(x_r).p_k,
  at every global-step boundary.
* Receiver injection (backward run): the recorded data are linear in time
  between global-step samples and zero after t_f.
* Ricker wavelet: (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - t_p.
"""
from __future__ import annotations

import numpy as np

from .mesh import OMesh


def ricker(t, f_peak: float, t_peak: float, amp: float = 1.0):
    a = (np.pi * f_peak * (np.asarray(t) - t_peak)) ** 2
    return amp * (1.0 - 2.0 * a) * np.exp(-a)


def barycentric(mesh: OMesh, k: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Barycentric coordinates (n,4) of points x (n,3) in elements k (n,)."""
    v = mesh.verts[mesh.etov[k]]                  # (n,4,3)
    T = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)
    lam123 = np.linalg.solve(T, (x - v[:, 0])[:, :, None])[:, :, 0]
    return np.concatenate([1.0 - lam123.sum(1, keepdims=True), lam123], axis=1)


def locate(mesh: OMesh, pts: np.ndarray, tol: float = 1e-12) -> np.ndarray:
    """Lowest element index containing each point (bucket search on element bounding boxes)."""
    pts = np.atleast_2d(pts)
    v = mesh.verts[mesh.etov]
    lo, hi = v.min(1), v.max(1)
    out = np.full(pts.shape[0], -1, dtype=np.int64)
    for i, x in enumerate(pts):
        cand = np.nonzero(np.all((lo <= x + 1e-9) & (hi >= x - 1e-9), axis=1))[0]
        if cand.size == 0:
            continue
        lam = barycentric(mesh, cand, np.repeat(x[None], cand.size, 0))
        ok = cand[np.all(lam >= -tol, axis=1)]
        if ok.size:
            out[i] = ok.min()
    if np.any(out < 0):
        raise ValueError("point outside the mesh")
    return out


def reference_coords(mesh: OMesh, k: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(r,s,t) of points x in elements k, from the barycentric coordinates."""
    lam = barycentric(mesh, k, x)
    return 2.0 * lam[:, 1:4] - 1.0


def interp_rows(mesh: OMesh, k: np.ndarray, x: np.ndarray) -> np.ndarray:
    """l(x_r): (n, Np) Lagrange values evaluating a field of element k at x."""
    return mesh.ref.lagrange_at(reference_coords(mesh, k, x))


def delta_weights(mesh: OMesh, k: np.ndarray, x: np.ndarray) -> np.ndarray:
    """w = M_k^{-1} l(x0) = (1/J_k) M_ref^{-1} l(r0): (n, Np)."""
    l = interp_rows(mesh, k, x)
    return (l @ mesh.ref.Minv.T) / mesh.J[k][:, None]


def data_at(data: np.ndarray, n_local: int, j: int) -> np.ndarray:
    """Receiver data (n_rec, n_t), sampled every global step (n_local local steps), at
    physical time j*dt_local: linear between samples, zero after the last sample."""
    n_t = data.shape[1]
    g, rem = divmod(j, n_local)
    if j < 0 or g > n_t - 1 or (g == n_t - 1 and rem > 0):
        return np.zeros(data.shape[0])
    if rem == 0:
        return data[:, g].astype(np.float64)
    th = rem / n_local
    return (1.0 - th) * data[:, g] + th * data[:, g + 1]
