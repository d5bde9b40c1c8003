"""FP64 reference tetrahedron for the nodal DG oracle.

TEST INFRASTRUCTURE ONLY.  Nothing under oracle/ is part of the product path;
only tests, the smoke check and the benchmark's CPU-baseline leg may import it.

Follows the nodal-DG section (Lagrange basis on warp-and-blend nodes,
Np = (N+1)(N+2)(N+3)/6) and the appendix (mass, stiffness and face-mass
matrices; D_j and L_f obtained by inverting the mass matrix).

Deliberately plain: the polynomial space is spanned by monomials
r^a s^b t^c (a+b+c <= N); every integral of a product of monomials over the
reference tetrahedron or a reference face is evaluated exactly with Python
fractions; the small dense algebra on top (Vandermonde inverse, products,
mass-matrix inverse) runs in 40-digit mpmath and is rounded once to FP64.
This is slow and obviously correct, and shares nothing with the library's
orthonormal-basis construction.

Reference tetrahedron: vertices V0=(-1,-1,-1), V1=(1,-1,-1), V2=(-1,1,-1),
V3=(-1,-1,1).  Faces, numbered 0..3: t=-1 (V0,V1,V2), s=-1 (V0,V1,V3),
r+s+t=-1 (V1,V2,V3), r=-1 (V0,V2,V3).  Node (i,j,l) with i+j+l <= N has
integer barycentric weights (N-i-j-l, i, j, l) on (V0,V1,V2,V3); nodes are
ordered with l slowest, then j, then i fastest.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb, factorial

import mpmath
import numpy as np

FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))
# the two reference coordinates that stay free on each face (r=0, s=1, t=2)
FACE_FREE = ((0, 1), (0, 2), (0, 1), (1, 2))

# Warp-and-blend optimised blending parameter alpha_opt for N = 1..15 (Warburton 2006, table of
# optimised 3-D alpha values).  Only N <= 6 is used here.
ALPHA_OPT = (0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577, 1.1603, 1.10153,
             0.6080, 0.4523, 0.8856, 0.8717, 0.9655)


def n_nodes(N: int) -> int:
    return (N + 1) * (N + 2) * (N + 3) // 6


def n_face_nodes(N: int) -> int:
    return (N + 1) * (N + 2) // 2


def lattice(N: int) -> np.ndarray:
    """(Np, 4) integer barycentric weights, in node order."""
    out = []
    for l in range(N + 1):
        for j in range(N + 1 - l):
            for i in range(N + 1 - l - j):
                out.append((N - i - j - l, i, j, l))
    return np.array(out, dtype=np.int64)


def gauss_lobatto(N: int) -> np.ndarray:
    """Legendre-Gauss-Lobatto points on [-1,1]: the end points and the roots of P_N'."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = np.sort(np.polynomial.legendre.Legendre.basis(N).deriv().roots().real)
    return np.concatenate([[-1.0], inner, [1.0]])


def _scaled_warp(N: int, r: np.ndarray) -> np.ndarray:
    """w(r)/(1-r^2), with w the 1-D warp mapping N+1 equispaced points onto the LGL points.

    w(r) = sum_i (x_LGL_i - x_eq_i) * lagrange_eq_i(r).  The end-point terms vanish
    (both sets contain -1 and 1), and for interior i the factor (r+1)(r-1) of
    lagrange_eq_i cancels the (1-r^2) analytically.
    """
    xeq = np.linspace(-1.0, 1.0, N + 1)
    xgl = gauss_lobatto(N)
    out = np.zeros_like(r)
    for i in range(1, N):
        term = np.full_like(r, (xgl[i] - xeq[i]) / (1.0 - xeq[i] ** 2))
        for j in range(1, N):
            if j != i:
                term = term * (r - xeq[j]) / (xeq[i] - xeq[j])
        out += term
    return out


_EQUI = np.array([[-1.0, -1.0 / np.sqrt(3.0), -1.0 / np.sqrt(6.0)],
                  [1.0, -1.0 / np.sqrt(3.0), -1.0 / np.sqrt(6.0)],
                  [0.0, 2.0 / np.sqrt(3.0), -1.0 / np.sqrt(6.0)],
                  [0.0, 0.0, 3.0 / np.sqrt(6.0)]])   # equilateral tetrahedron, edge length 2


def warp_blend_nodes(N: int) -> np.ndarray:
    """(Np, 3) reference coordinates (r,s,t) of the warp-and-blend nodes (Warburton 2006).

    Built on the equilateral tetrahedron: each face contributes the 2-D warp of its
    three edges (edge warp along the edge, blended by 4*L_i*L_j*(1+(alpha*L_opp)^2)),
    and the face warps are blended into the interior by
    L_b L_c L_d / prod(L_x + L_a/2) * (1+(alpha*L_a)^2).  Nodes lying on an edge take
    the face warp directly (the 3-D blend is 0/0 there).
    """
    alpha = ALPHA_OPT[N - 1] if N >= 1 else 0.0
    lam = lattice(N).astype(np.float64) / N if N > 0 else np.array([[1.0, 0, 0, 0]])
    X = lam @ _EQUI
    shift = np.zeros_like(X)
    tol = 1e-10
    faces = ((0, (1, 2, 3)), (1, (0, 2, 3)), (2, (0, 1, 3)), (3, (0, 1, 2)))
    for a, (b, c, d) in faces:
        La = lam[:, a]
        fw = np.zeros_like(X)
        for (i, j, o) in ((b, c, d), (c, d, b), (d, b, c)):
            r = lam[:, j] - lam[:, i]
            u = (_EQUI[j] - _EQUI[i]) / 2.0
            amp = 4.0 * lam[:, i] * lam[:, j] * _scaled_warp(N, r) * (1.0 + (alpha * lam[:, o]) ** 2)
            fw += amp[:, None] * u[None, :]
        Lb, Lc, Ld = lam[:, b], lam[:, c], lam[:, d]
        blend = Lb * Lc * Ld
        denom = (Lb + 0.5 * La) * (Lc + 0.5 * La) * (Ld + 0.5 * La)
        ok = denom > tol
        blend = np.where(ok, (1.0 + (alpha * La) ** 2) * blend / np.where(ok, denom, 1.0), blend)
        shift += blend[:, None] * fw
        on_edge = (La < tol) & (((Lb > tol).astype(int) + (Lc > tol) + (Ld > tol)) < 3)
        shift[on_edge] = fw[on_edge]
    X = X + shift
    # back to barycentric coordinates on the equilateral tet, then to (r,s,t)
    A = np.vstack([_EQUI.T, np.ones(4)])
    mu = np.linalg.solve(A, np.vstack([X.T, np.ones(X.shape[0])])).T
    return 2.0 * mu[:, 1:4] - 1.0


# ----------------------------------------------------------------------------------------
# exact integrals of monomials
# ----------------------------------------------------------------------------------------

def monomials3(N: int) -> list[tuple[int, int, int]]:
    return [(a, b, c) for c in range(N + 1) for b in range(N + 1 - c) for a in range(N + 1 - b - c)]


def monomials2(N: int) -> list[tuple[int, int]]:
    return [(a, b) for b in range(N + 1) for a in range(N + 1 - b)]


def _shifted_coeffs(a: int):
    # (-1 + 2x)^a = sum_i comb(a,i) 2^i (-1)^(a-i) x^i
    return [(i, Fraction(comb(a, i) * 2 ** i * (-1) ** (a - i))) for i in range(a + 1)]


@lru_cache(maxsize=None)
def tet_monomial_integral(a: int, b: int, c: int) -> Fraction:
    """Exact integral of r^a s^b t^c over the reference tetrahedron."""
    tot = Fraction(0)
    for i, ci in _shifted_coeffs(a):
        for j, cj in _shifted_coeffs(b):
            for k, ck in _shifted_coeffs(c):
                tot += ci * cj * ck * Fraction(factorial(i) * factorial(j) * factorial(k),
                                               factorial(i + j + k + 3))
    return 8 * tot


@lru_cache(maxsize=None)
def tri_monomial_integral(a: int, b: int) -> Fraction:
    """Exact integral of u^a v^b over the reference triangle {u,v >= -1, u+v <= 0} (area 2)."""
    tot = Fraction(0)
    for i, ci in _shifted_coeffs(a):
        for j, cj in _shifted_coeffs(b):
            tot += ci * cj * Fraction(factorial(i) * factorial(j), factorial(i + j + 2))
    return 4 * tot


def _mpq(x: Fraction):
    return mpmath.mpf(x.numerator) / x.denominator


def _mp_vander3(pts, mons, deriv=None):
    """Monomial (or monomial-derivative) Vandermonde in mpmath at the FP64 points."""
    rows = []
    for p in pts:
        r, s, t = (mpmath.mpf(float(x)) for x in p)
        row = []
        for e in mons:
            e = list(e)
            coef = 1
            if deriv is not None:
                coef = e[deriv]
                if coef == 0:
                    row.append(mpmath.mpf(0))
                    continue
                e[deriv] -= 1
            row.append(coef * r ** e[0] * s ** e[1] * t ** e[2])
        rows.append(row)
    return mpmath.matrix(rows)


def _to_np(A) -> np.ndarray:
    return np.array([[float(A[i, j]) for j in range(A.cols)] for i in range(A.rows)])


def _vander3(pts: np.ndarray, mons, deriv: int | None = None) -> np.ndarray:
    r, s, t = pts[:, 0], pts[:, 1], pts[:, 2]
    V = np.zeros((pts.shape[0], len(mons)))
    for p, e in enumerate(mons):
        e = list(e)
        coef = 1.0
        if deriv is not None:
            coef = float(e[deriv])
            if e[deriv] == 0:
                continue
            e[deriv] -= 1
        V[:, p] = coef * r ** e[0] * s ** e[1] * t ** e[2]
    return V


class RefElement:
    """Operators of the order-N reference tetrahedron.

    The dense algebra (Vandermonde inverse, products, mass-matrix inverse) is
    done in 40-digit mpmath arithmetic on the FP64 node coordinates and rounded
    once to FP64, because the monomial basis is ill-conditioned at N = 6.
    """

    def __init__(self, N: int):
        self.N = N
        self.Np = n_nodes(N)
        self.Nfp = n_face_nodes(N)
        self.lat = lattice(N)
        self.rst = warp_blend_nodes(N)
        mons = monomials3(N)
        self.mons = mons
        with mpmath.workdps(40):
            V = _mp_vander3(self.rst, mons)
            Vi = V ** -1
            Dr = _mp_vander3(self.rst, mons, 0) * Vi
            Ds = _mp_vander3(self.rst, mons, 1) * Vi
            Dt = _mp_vander3(self.rst, mons, 2) * Vi
            G = mpmath.matrix([[_mpq(tet_monomial_integral(a1 + a2, b1 + b2, c1 + c2)) for (a2, b2, c2) in mons]
                               for (a1, b1, c1) in mons])
            M = Vi.T * G * Vi
            Mi = M ** -1
            opp = (3, 2, 0, 1)
            self.Fmask = np.array([np.nonzero(self.lat[:, opp[f]] == 0)[0] for f in range(4)])
            mons2 = monomials2(N)
            G2 = mpmath.matrix([[_mpq(tri_monomial_integral(a1 + a2, b1 + b2)) for (a2, b2) in mons2]
                                for (a1, b1) in mons2])
            E = mpmath.zeros(self.Np, 4 * self.Nfp)
            self.Mface = []
            for f in range(4):
                uv = self.rst[self.Fmask[f]][:, list(FACE_FREE[f])]
                Vf = mpmath.matrix([[mpmath.mpf(float(u)) ** a * mpmath.mpf(float(v)) ** b for (a, b) in mons2]
                                    for (u, v) in uv])
                Vfi = Vf ** -1
                Mf = Vfi.T * G2 * Vfi
                self.Mface.append(_to_np(Mf))
                for i, n in enumerate(self.Fmask[f]):
                    for j in range(self.Nfp):
                        E[int(n), f * self.Nfp + j] = Mf[i, j]
            L = Mi * E
            self.V, self.Vinv = _to_np(V), _to_np(Vi)
            self.Dr, self.Ds, self.Dt = _to_np(Dr), _to_np(Ds), _to_np(Dt)
            self.M, self.Minv = _to_np(M), _to_np(Mi)
            self.E, self.LIFT = _to_np(E), _to_np(L)

    def lagrange_at(self, rst: np.ndarray) -> np.ndarray:
        """Values of the Np Lagrange basis functions at points rst (n,3) -> (n, Np)."""
        return _vander3(np.atleast_2d(rst), self.mons) @ self.Vinv


@lru_cache(maxsize=None)
def get_ref(N: int) -> RefElement:
    """Cached reference element of order N."""
    return RefElement(N)
