"""Pins of the oracle's reference element against mathematics and the paper's printed values."""
import json
import os
from fractions import Fraction
from itertools import permutations

import numpy as np
import pytest
from scipy import integrate

from oracle.refelem import RefElement, gauss_lobatto, n_nodes, warp_blend_nodes, FACE_FREE
from oracle import timestep as T

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


@pytest.fixture(scope="module", params=[1, 2, 3, 4, 5, 6])
def ref(request):
    return RefElement(request.param)


def test_np_formula_and_dof_identity():
    g = GOLD["np_formula"]
    assert [n_nodes(N) for N in g["N"]] == g["Np"]
    d = GOLD["dof_identity"]
    assert d["K"] * n_nodes(d["N"]) * d["fields"] == d["dof"]


def test_ab_coefficients_match_paper():
    a, b, ebar, C, Cmix = T.ab_coefficients()
    g = GOLD["ab3_a"]
    assert a == [Fraction(x, g["den"]) for x in g["num"]]
    g = GOLD["ab3_b_half_step"]
    assert b == [Fraction(x, g["den"]) for x in g["num"]]
    assert C == [[Fraction(x) for x in row] for row in GOLD["image_C"]["rows"]]
    # the dt^2 weights of the exact correlation must be int_0^1 A_s, not a_s (garble of the printed formula)
    assert ebar == [Fraction(19, 24), Fraction(-5, 12), Fraction(1, 8)]
    # constant rhs: sums are int_0^1 theta = 1/2, int theta^2 = 1/3, int theta (1-theta) = 1/6
    assert sum(ebar) == Fraction(1, 2)
    assert sum(sum(r) for r in C) == Fraction(1, 3)
    assert sum(sum(r) for r in Cmix) == Fraction(1, 6)


def test_ab_coefficients_by_quadrature():
    # exactness of AB3 on quadratic rhs: integrate l_s numerically
    from numpy.polynomial import polynomial as P
    a, b, *_ = T.ab_coefficients()
    for s in range(3):
        nodes = [0, -1, -2]
        others = [x for i, x in enumerate(nodes) if i != s]
        f = lambda th: np.prod([(th - x) / (nodes[s] - x) for x in others])
        assert abs(integrate.quad(f, 0, 1)[0] - float(a[s])) < 1e-14
        assert abs(integrate.quad(f, 0, 0.5)[0] - float(b[s])) < 1e-14


def test_lgl_edges(ref):
    N = ref.N
    r = ref.rst
    for (i, j) in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)):
        on = np.nonzero(np.all(np.delete(ref.lat, [i, j], axis=1) == 0, axis=1))[0]
        # coordinate along the edge from barycentric weights
        V = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
        d = V[j] - V[i]
        u = (r[on] - V[i]) @ d / (d @ d) * 2 - 1
        assert np.allclose(np.sort(u), gauss_lobatto(N), atol=1e-14)


def test_node_set_symmetric(ref):
    # the node set is invariant under every relabelling of the 4 vertices
    V = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    lam = np.concatenate([-(1 + ref.rst.sum(1, keepdims=True)) / 2, (1 + ref.rst) / 2], axis=1)
    base = {tuple(np.round(x, 12)) for x in lam @ V}
    for p in permutations(range(4)):
        pts = lam[:, list(p)] @ V
        assert {tuple(np.round(x, 12)) for x in pts} == base


def test_mass_matrix_integrates_polynomials(ref):
    # 1^T M f = integral of f over the reference tet, checked with scipy's adaptive quadrature
    r, s, t = ref.rst.T
    N = ref.N
    funcs = [lambda r, s, t: 1.0 + 0 * r, lambda r, s, t: r * s ** 2 if N >= 3 else r,
             lambda r, s, t: (t + 0.3) ** N]
    for f in funcs:
        val = ref.M.sum(0) @ f(r, s, t)
        ex = integrate.tplquad(lambda tt, ss, rr: f(rr, ss, tt), -1, 1, lambda rr: -1, lambda rr: -rr,
                               lambda rr, ss: -1, lambda rr, ss: -1 - rr - ss, epsabs=1e-13, epsrel=1e-13)[0]
        assert abs(val - ex) < 1e-11 * max(1, abs(ex))


def test_exact_differentiation(ref):
    rng = np.random.default_rng(ref.N)
    r, s, t = ref.rst.T
    N = ref.N
    for _ in range(3):
        a = rng.integers(0, N + 1)
        b = rng.integers(0, N + 1 - a)
        c = rng.integers(0, N + 1 - a - b)
        f = r ** a * s ** b * t ** c
        dr = a * r ** max(a - 1, 0) * s ** b * t ** c
        ds = b * r ** a * s ** max(b - 1, 0) * t ** c
        dt = c * r ** a * s ** b * t ** max(c - 1, 0)
        for D, ex in ((ref.Dr, dr), (ref.Ds, ds), (ref.Dt, dt)):
            assert np.abs(D @ f - ex).max() < 1e-10 * max(1.0, np.abs(ex).max())


def test_integration_by_parts_pins_M_D_and_face_mass(ref):
    # M D_j + (M D_j)^T = sum_f nraw_{f,j} E_f E_f^T-embedded face mass (divergence theorem on the
    # reference tet; faces parameterised by their two free coordinates, nraw the unscaled normal)
    nraw = np.array([[0, 0, -1], [0, -1, 0], [1, 1, 1], [-1, 0, 0]], float)
    for j, D in enumerate((ref.Dr, ref.Ds, ref.Dt)):
        lhs = ref.M @ D + (ref.M @ D).T
        rhs = np.zeros_like(lhs)
        for f in range(4):
            idx = ref.Fmask[f]
            rhs[np.ix_(idx, idx)] += nraw[f, j] * ref.Mface[f]
        assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(lhs).max()


def test_lift_is_minv_times_face_mass(ref):
    # LIFT maps a face-node vector to M^{-1} * (face mass * vector); check on ones: sum of columns of
    # face f in M LIFT = face area 2 in the parameter plane
    ML = ref.M @ ref.LIFT
    for f in range(4):
        assert abs(ML[:, f * ref.Nfp:(f + 1) * ref.Nfp].sum() - 2.0) < 1e-10
