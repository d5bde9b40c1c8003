"""Seeded synthetic inputs: tetrahedral meshes, velocity models, shot geometry, request streams.

This module is the one place both the GPU library's callers and the FP64
oracle take their inputs from.  It holds no discontinuous-Galerkin
arithmetic: it only builds vertex coordinates, element-to-vertex lists,
per-element material values, point positions and arrival times.

The paper's own meshes and velocity models (the two-layer validation cube of
the validation section and the salt-dome mesh of the RTM section) are not
available, so the generators below stand in for them with the same shapes:
a planar dipping interface between a 1.5 km/s and a 3.0 km/s medium, a
source a few metres below the surface, a receiver grid at 10 m depth, and
meshes refined near interfaces so that multi-rate levels appear.

Meshes ("Kuhn boxes"): a logical nx*ny*nz grid of cells, each split into six
tetrahedra along its main diagonal, one per permutation of the three axes
(in itertools.permutations order).  Cells are numbered x fastest, then y,
then z; element id = 6*cell + permutation index.  The triangulation is
conforming because every cell uses the same split.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Mesh", "kuhn_box", "graded_layers", "unit_cube_mesh", "two_layer_mesh",
    "two_layer_model", "smooth_random_model", "receiver_grid", "ricker_peak_time",
    "poisson_arrivals", "ShotSpec", "config_mesh",
]

PERMS = list(itertools.permutations((0, 1, 2)))


@dataclass
class Mesh:
    """A tetrahedral mesh as plain arrays (user element order)."""
    verts: np.ndarray            # (n_vert, 3) float64
    etov: np.ndarray             # (K, 4) int64
    box: tuple                   # (Lx, Ly, Lz)
    meta: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return int(self.etov.shape[0])


def graded_layers(z0: float, z1: float, n: int, fine: list[tuple]) -> np.ndarray:
    """n+1 layer positions on [z0, z1]; cells inside a `fine` interval (a, b) get half thickness,
    inside (a, b, w) 1/w of the thickness.

    The positions are the inverse of the cumulative of a weight that is w (default 2) in the
    fine intervals and 1 elsewhere, sampled at n equal steps.
    """
    fine = [tuple(f) if len(f) == 3 else (f[0], f[1], 2.0) for f in fine]
    # breakpoints of the piecewise-constant weight
    pts = {z0, z1}
    for a, b, _ in fine:
        pts.add(min(max(a, z0), z1))
        pts.add(min(max(b, z0), z1))
    pts = np.array(sorted(pts))
    mids = 0.5 * (pts[:-1] + pts[1:])
    w = np.ones_like(mids)
    for a, b, wf in fine:
        w[(mids > a) & (mids < b)] = float(wf)
    cum = np.concatenate([[0.0], np.cumsum(w * np.diff(pts))])
    target = np.linspace(0.0, cum[-1], n + 1)
    idx = np.clip(np.searchsorted(cum, target, side="right") - 1, 0, len(w) - 1)
    z = pts[idx] + (target - cum[idx]) / w[idx]
    z[0], z[-1] = z0, z1
    return z


def kuhn_box(xs: np.ndarray, ys: np.ndarray, zcol) -> tuple[np.ndarray, np.ndarray]:
    """Vertices and element-to-vertex lists of a Kuhn-split box.

    xs (nx+1,), ys (ny+1,) are the x and y vertex positions; zcol(i) returns the
    nz+1 z positions of the vertex column at x index i (columns may differ in z).
    """
    nx, ny = len(xs) - 1, len(ys) - 1
    zc = np.stack([np.asarray(zcol(i), dtype=np.float64) for i in range(nx + 1)])  # (nx+1, nz+1)
    nz = zc.shape[1] - 1
    I, J, M = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    # vertex id = i + (nx+1)*(j + (ny+1)*m)
    verts = np.zeros(((nx + 1) * (ny + 1) * (nz + 1), 3))
    vid = I + (nx + 1) * (J + (ny + 1) * M)
    verts[vid.ravel(), 0] = xs[I.ravel()]
    verts[vid.ravel(), 1] = ys[J.ravel()]
    verts[vid.ravel(), 2] = zc[I.ravel(), M.ravel()]

    ci, cj, cm = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # cell id: x fastest, then y, then z
    ci, cj, cm = (a.transpose(2, 1, 0).ravel() for a in (ci, cj, cm))
    ncell = ci.size

    def v(di, dj, dm):
        return (ci + di) + (nx + 1) * ((cj + dj) + (ny + 1) * (cm + dm))

    etov = np.zeros((ncell, 6, 4), dtype=np.int64)
    for p, (a, b, _) in enumerate(PERMS):
        d0 = [0, 0, 0]
        d1 = list(d0); d1[a] = 1
        d2 = list(d1); d2[b] = 1
        etov[:, p, 0] = v(*d0)
        etov[:, p, 1] = v(*d1)
        etov[:, p, 2] = v(*d2)
        etov[:, p, 3] = v(1, 1, 1)
    return verts, etov.reshape(-1, 4)


def _orient(verts: np.ndarray, etov: np.ndarray) -> np.ndarray:
    """Swap local vertices 2 and 3 of every element whose signed volume is negative."""
    a = verts[etov[:, 1]] - verts[etov[:, 0]]
    b = verts[etov[:, 2]] - verts[etov[:, 0]]
    c = verts[etov[:, 3]] - verts[etov[:, 0]]
    det = np.einsum("ij,ij->i", a, np.cross(b, c))
    out = etov.copy()
    neg = det < 0
    out[neg, 2], out[neg, 3] = etov[neg, 3], etov[neg, 2]
    return out


def _jitter(verts, box, hx, hy, hz_of_vertex, rng, amp, fixed_z_fn=None, on_surface=None):
    """Move vertices by U(-amp, amp) * local spacing per coordinate.

    Boundary vertices only move tangentially to their boundary face(s).
    Vertices flagged `on_surface` get z re-projected onto fixed_z_fn(x) after
    the move so the mesh keeps conforming to that surface.
    """
    Lx, Ly, Lz = box
    n = verts.shape[0]
    d = rng.uniform(-amp, amp, size=(n, 3))
    d[:, 0] *= hx
    d[:, 1] *= hy
    d[:, 2] *= hz_of_vertex
    tol = 1e-12
    x, y, z = verts[:, 0], verts[:, 1], verts[:, 2]
    d[(np.abs(x) < tol) | (np.abs(x - Lx) < tol), 0] = 0.0
    d[(np.abs(y) < tol) | (np.abs(y - Ly) < tol), 1] = 0.0
    d[(np.abs(z) < tol) | (np.abs(z - Lz) < tol), 2] = 0.0
    out = verts + d
    if on_surface is not None and fixed_z_fn is not None:
        out[on_surface, 2] = fixed_z_fn(out[on_surface, 0])
    return out


def _vertex_dz(zc_of_vertex_layers: np.ndarray, layer: np.ndarray, col: np.ndarray) -> np.ndarray:
    """Local z spacing at a vertex: the thinner of its two adjacent cells in its column."""
    zc = zc_of_vertex_layers
    nz = zc.shape[1] - 1
    below = np.where(layer > 0, zc[col, np.maximum(layer, 1)] - zc[col, np.maximum(layer - 1, 0)], np.inf)
    above = np.where(layer < nz, zc[col, np.minimum(layer + 1, nz)] - zc[col, np.minimum(layer, nz - 1)], np.inf)
    return np.minimum(below, above)


def unit_cube_mesh(n: int = 8) -> Mesh:
    """Unit cube, n^3 cells x 6 tetrahedra, no jitter (the eigenmode box)."""
    g = np.linspace(0.0, 1.0, n + 1)
    verts, etov = kuhn_box(g, g, lambda i: g)
    etov = _orient(verts, etov)
    return Mesh(verts, etov, (1.0, 1.0, 1.0), {"kind": "unit_cube", "n": n})


def _interface_depth(x, d0, slope):
    return d0 + slope * x


def two_layer_mesh(nx: int, ny: int, nz: int, box=(2.0, 2.0, 1.0), d0=0.35, slope=0.15,
                   band=0.1, jitter=0.1, seed=1234) -> Mesh:
    """Box with z up and the top surface at z = Lz, conforming to a dipping plane.

    The interface sits at depth d(x) = d0 + slope*x.  One vertex layer (index
    n_below) lies exactly on it in every column; cells within `band` of it get
    half thickness.  Interior vertices are jittered by U(-jitter, jitter) times
    the local spacing with a seeded PCG64 generator.
    """
    Lx, Ly, Lz = box
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = np.linspace(0.0, Ly, ny + 1)

    def zi(x):
        return Lz - _interface_depth(x, d0, slope)

    # split of the nz layers between below/above, fixed from the middle column
    zm = zi(0.5 * Lx)
    wb = zm + min(band, zm)
    wa = (Lz - zm) + min(band, Lz - zm)
    n_below = int(round(nz * wb / (wa + wb)))
    n_below = min(max(n_below, 1), nz - 1)
    n_above = nz - n_below

    def zcol(i):
        z_int = zi(xs[i])
        lo = graded_layers(0.0, z_int, n_below, [(z_int - band, z_int)])
        hi = graded_layers(z_int, Lz, n_above, [(z_int, z_int + band)])
        return np.concatenate([lo, hi[1:]])

    verts, etov = kuhn_box(xs, ys, zcol)
    zc = np.stack([zcol(i) for i in range(nx + 1)])
    nv = verts.shape[0]
    vid = np.arange(nv)
    col = vid % (nx + 1)
    layer = vid // ((nx + 1) * (ny + 1))
    hz = _vertex_dz(zc, layer, col)
    rng = np.random.default_rng(seed)
    on_if = layer == n_below
    verts = _jitter(verts, box, Lx / nx, Ly / ny, hz, rng, jitter,
                    fixed_z_fn=zi, on_surface=on_if)
    etov = _orient(verts, etov)
    meta = {"kind": "two_layer", "nx": nx, "ny": ny, "nz": nz, "d0": d0, "slope": slope,
            "n_below": n_below, "seed": seed, "jitter": jitter, "band": band}
    return Mesh(verts, etov, box, meta)


def centroids(mesh: Mesh) -> np.ndarray:
    return mesh.verts[mesh.etov].mean(axis=1)


def two_layer_model(mesh: Mesh, c_top=1.5, c_bottom=3.0, rho=1.0):
    """Per-element (rho, c): c_top above the dipping plane, c_bottom below (centroid rule)."""
    Lz = mesh.box[2]
    xc = centroids(mesh)
    zi = Lz - _interface_depth(xc[:, 0], mesh.meta["d0"], mesh.meta["slope"])
    c = np.where(xc[:, 2] > zi, c_top, c_bottom).astype(np.float64)
    return np.full(mesh.K, float(rho)), c


def graded_top_mesh(nx, ny, nz, box=(10.0, 10.0, 4.0), top=0.5, refine=4.0, jitter=0.1, seed=5) -> Mesh:
    """Box whose top `top` km has cells 1/refine as thick as below (the largest single-GPU shot:
    with refine = 4 and velocities over a 3x range the element time steps span more than 8x,
    hence four LTS levels)."""
    Lx, Ly, Lz = box
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = np.linspace(0.0, Ly, ny + 1)
    zl = graded_layers(0.0, Lz, nz, [(Lz - top, Lz, refine)])
    verts, etov = kuhn_box(xs, ys, lambda i: zl)
    zc = np.tile(zl, (nx + 1, 1))
    nv = verts.shape[0]
    vid = np.arange(nv)
    hz = _vertex_dz(zc, vid // ((nx + 1) * (ny + 1)), vid % (nx + 1))
    rng = np.random.default_rng(seed)
    verts = _jitter(verts, box, Lx / nx, Ly / ny, hz, rng, jitter)
    etov = _orient(verts, etov)
    return Mesh(verts, etov, box, {"kind": "graded_top", "nx": nx, "ny": ny, "nz": nz, "seed": seed})


def smooth_random_model(mesh: Mesh, seed=5, grid=0.1, sigma=0.5, cmin=1.5, cmax=4.5,
                        ellipsoid=((5.0, 5.0), 2.0, (2.0, 1.5, 0.6), 4.5), rho=1.0):
    """Gaussian-filtered seeded noise rescaled to [cmin, cmax] plus a fast ellipsoid."""
    from scipy.ndimage import gaussian_filter
    Lx, Ly, Lz = mesh.box
    shape = tuple(int(math.ceil(L / grid)) + 1 for L in (Lx, Ly, Lz))
    rng = np.random.default_rng(seed)
    noise = gaussian_filter(rng.standard_normal(shape), sigma / grid, mode="nearest")
    lo, hi = noise.min(), noise.max()
    field_ = cmin + (cmax - cmin) * (noise - lo) / (hi - lo)
    xc = centroids(mesh)
    idx = np.clip(np.rint(xc / grid).astype(np.int64), 0, np.array(shape) - 1)
    c = field_[idx[:, 0], idx[:, 1], idx[:, 2]]
    (ex, ey), depth, (ax, ay, az), c_e = ellipsoid
    ez = Lz - depth
    inside = (((xc[:, 0] - ex) / ax) ** 2 + ((xc[:, 1] - ey) / ay) ** 2 + ((xc[:, 2] - ez) / az) ** 2) <= 1.0
    c = np.where(inside, c_e, c)
    return np.full(mesh.K, float(rho)), c.astype(np.float64)


def receiver_grid(n: int, lo: float, hi: float, z: float) -> np.ndarray:
    """n*n receivers on [lo, hi]^2 at height z (x fastest)."""
    g = np.linspace(lo, hi, n)
    X, Y = np.meshgrid(g, g, indexing="xy")
    return np.stack([X.ravel(), Y.ravel(), np.full(n * n, z)], axis=1)


def ricker_peak_time(f_peak: float) -> float:
    """Peak time of the Ricker wavelet: the paper's 0.1127 s, later if the pulse is wider."""
    return max(0.1127, 1.5 / f_peak)


def poisson_arrivals(n: int, rate: float, seed: int = 7) -> np.ndarray:
    """n arrival times of a Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


@dataclass
class ShotSpec:
    src: np.ndarray              # (3,)
    f_peak: float
    t_peak: float
    rec: np.ndarray              # (n_rec, 3)
    t_final: float
    amp: float = 1.0


def config_mesh(name: str) -> tuple[Mesh, np.ndarray, np.ndarray, int]:
    """(mesh, rho, c, N) for the named workload."""
    if name == "eigen_cube":          # 3072 tets, N=3, rho=c=1, rigid walls
        m = unit_cube_mesh(8)
        return m, np.ones(m.K), np.ones(m.K), 3
    if name == "eigen_cube_n6":
        m = unit_cube_mesh(8)
        return m, np.ones(m.K), np.ones(m.K), 6
    if name == "rtm_200k":            # 201600 tets, N=4
        m = two_layer_mesh(40, 40, 21, seed=1234)
        rho, c = two_layer_model(m)
        return m, rho, c, 4
    if name == "rtm_200k_n6":
        m = two_layer_mesh(40, 40, 21, seed=1234)
        rho, c = two_layer_model(m)
        return m, rho, c, 6
    if name == "srv_50k":
        m = two_layer_mesh(26, 26, 13, seed=101)
        rho, c = two_layer_model(m)
        return m, rho, c, 3
    if name == "srv_200k":
        m = two_layer_mesh(40, 40, 21, seed=102)
        rho, c = two_layer_model(m)
        return m, rho, c, 4
    if name == "srv_800k":
        m = two_layer_mesh(64, 64, 32, seed=103)
        rho, c = two_layer_model(m)
        return m, rho, c, 5
    if name == "big_4m":
        m = graded_top_mesh(120, 120, 48)
        rho, c = smooth_random_model(m)
        return m, rho, c, 4
    if name.startswith("two_layer_small"):  # small parity meshes: two_layer_small:nx:ny:nz:N
        _, nx, ny, nz, N = name.split(":")
        m = two_layer_mesh(int(nx), int(ny), int(nz), seed=42)
        rho, c = two_layer_model(m)
        return m, rho, c, int(N)
    raise KeyError(name)


def rtm_shot(box=(2.0, 2.0, 1.0), src_xy=(0.7797, 1.0), f_peak=15.0, n_rec=100, t_final=1.0) -> ShotSpec:
    """A surface shot: source 8 m deep, an n_rec x n_rec receiver grid 10 m deep."""
    Lx, Ly, Lz = box
    src = np.array([src_xy[0], src_xy[1], Lz - 0.008])
    step = Lx / n_rec
    rec = receiver_grid(n_rec, 0.5 * step, Lx - 0.5 * step, Lz - 0.010)
    return ShotSpec(src, f_peak, ricker_peak_time(f_peak), rec, t_final)
