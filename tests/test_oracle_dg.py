"""Pins of the oracle's mesh, DG operator and time integrators against mathematics."""
import numpy as np
import pytest

from oracle.dg import Operator
from oracle.mesh import BC_FREE, BC_RIGID, BC_TRANSPARENT, OMesh, local_dt, lts_levels
from oracle.refelem import get_ref
from oracle import timestep as T
from paper_1506_00907_amd import inputs as I
from tests.oracle_cases import case, eigenmode


def _mixed_bc_mesh(N=3, seed=3):
    m = I.two_layer_mesh(4, 4, 4, seed=seed)
    rho, c = I.two_layer_model(m)
    rng = np.random.default_rng(seed)
    rho = rho * rng.uniform(0.8, 1.6, m.K)          # heterogeneous impedance
    bc = rng.choice([BC_RIGID, BC_TRANSPARENT, BC_FREE], size=(m.K, 4))
    M = OMesh(get_ref(N), m.verts, m.etov, face_bc=bc)
    return M, Operator(M, rho, c)


def test_connectivity_invariants():
    m, op, *_ = case("two_layer_small:6:6:4:3")
    M = op.m
    k = np.arange(M.K)[:, None]
    inter = ~M.is_bdry
    assert np.all(M.EToE[M.EToE, M.EToF][inter] == np.broadcast_to(k, M.EToE.shape)[inter])
    xM = M.x.reshape(-1, 3)[M.vmapM]
    xP = M.x.reshape(-1, 3)[M.vmapP]
    assert np.abs(xM - xP).max() < 1e-13
    # boundary faces lie on the box faces
    Lx, Ly, Lz = m.box
    fb = M.x[np.nonzero(M.is_bdry)[0]]
    assert M.is_bdry.sum() == 2 * 2 * (6 * 6 + 6 * 4 + 6 * 4)


def test_geometry():
    m, op, *_ = case("two_layer_small:6:6:4:3")
    M = op.m
    assert abs(M.volume.sum() - 4.0) < 1e-12
    # closed surface: sum_f |face| n_f = 0, with |face| = 2 sJ in the parameter plane
    s = np.einsum("kf,kfd->kd", M.sJ, M.n)
    assert np.abs(s).max() < 1e-12
    # outward: normal points from element centroid to face centroid
    cen = M.verts[M.etov].mean(1)
    from oracle.refelem import FACE_VERTS
    for f, fv in enumerate(FACE_VERTS):
        fc = M.verts[M.etov[:, list(fv)]].mean(1)
        assert np.all(np.einsum("kd,kd->k", fc - cen, M.n[:, f]) > 0)


@pytest.mark.parametrize("N", [1, 3, 4])
def test_physical_derivatives_exact_on_random_affine_tet(N):
    # pins the reading g^vol = dr_j/dx_i (inverse Jacobian): the chain rule must be exact
    rng = np.random.default_rng(N)
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) + 0.2 * rng.standard_normal((4, 3))
    M = OMesh(get_ref(N), verts, np.array([[0, 1, 2, 3]]))
    x, y, z = M.x[0].T
    R = M.ref
    c2 = 0.5 if N >= 2 else 0.0
    f = x ** N + c2 * x * y * z ** max(N - 2, 0) + y
    fx = N * x ** (N - 1) + c2 * y * z ** max(N - 2, 0)
    G = M.grad[0]
    dfdx = sum(G[j, 0] * (D @ f) for j, D in enumerate((R.Dr, R.Ds, R.Dt)))
    assert np.abs(dfdx - fx).max() < 1e-11 * np.abs(fx).max()


def test_central_flux_is_skew_and_needs_the_half():
    # with tau = 0 and rigid walls, q^T W rhs(q) = 0 (energy-conserving); W = blockdiag(J M/(rho c^2), J rho M)
    M, op = _mixed_bc_mesh()
    op.m.bc[op.m.is_bdry] = BC_RIGID
    rng = np.random.default_rng(1)
    q = rng.standard_normal((M.K, 4, M.ref.Np))
    r = op.rhs(q, tau_sign=0.0)
    W = _wdot(op, q, r)
    assert abs(W) < 1e-12 * np.sqrt(_wdot(op, q, q) * _wdot(op, r, r))


def _wdot(op, a, b):
    J, Mm = op.m.J, op.ref.M
    out = np.einsum("k,kn,nm,km->", J / (op.rho * op.c ** 2), a[:, 0], Mm, b[:, 0])
    for d in range(1, 4):
        out += np.einsum("k,kn,nm,km->", J * op.rho, a[:, d], Mm, b[:, d])
    return out


def test_energy_identity_upwind_heterogeneous_all_bcs():
    # q^T W rhs(q) = -1/2 sum_interior_faces int (tau_p [[p]]^2 + tau_v [[n.v]]^2)
    #               - sum_boundary: rigid tau_v (n.v)^2, transparent (tau_p p^2 + tau_v (n.v)^2)/2, free tau_p p^2
    M, op = _mixed_bc_mesh()
    rng = np.random.default_rng(2)
    q = rng.standard_normal((M.K, 4, M.ref.Np))
    lhs = _wdot(op, q, op.rhs(q))
    tr = op.traces(q)
    pM, nvM = tr[..., 0], tr[..., 1]
    pP = tr[M.EToE[:, :, None], M.EToF[:, :, None], M.nbr_node, 0]
    nvP = -tr[M.EToE[:, :, None], M.EToF[:, :, None], M.nbr_node, 1]
    rhs = 0.0
    for k in range(M.K):
        for f in range(4):
            Mf = M.ref.Mface[f] * M.sJ[k, f]
            quad = lambda a: a @ Mf @ a
            tp, tv = op.tau_p[k, f], op.tau_v[k, f]
            b = M.bc[k, f]
            if not M.is_bdry[k, f]:
                rhs += -0.25 * (tp * quad(pP[k, f] - pM[k, f]) + tv * quad(nvP[k, f] - nvM[k, f]))
            elif b == BC_RIGID:
                rhs += -tv * quad(nvM[k, f])
            elif b == BC_TRANSPARENT:
                rhs += -0.5 * (tp * quad(pM[k, f]) + tv * quad(nvM[k, f]))
            elif b == BC_FREE:
                rhs += -tp * quad(pM[k, f])
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)
    # backward in time with tau -> -tau is dissipative in reversed time as well
    assert _wdot(op, q, op.rhs_reversed(q)) < 0


def test_eigenmode_closed_form_lserk4_and_ab3():
    m, op, *_ = case("eigen_cube", bc=BC_RIGID)
    M = op.m
    dt = local_dt(M.verts, M.etov, op.c, 3).min()
    assert abs(dt - 8.2864e-4) < 1e-7                   # l = h/sqrt(2) for the Kuhn tet of side 1/8
    n = 25
    q0 = eigenmode(M, 0.0)
    e0 = np.sqrt(op.energy(q0))
    q1 = T.lserk4(op, q0, dt, n)
    err_rk = np.sqrt(op.energy(q1 - eigenmode(M, n * dt))) / e0
    h = np.stack([op.rhs(eigenmode(M, -dt)), op.rhs(eigenmode(M, -2 * dt))])
    q2, _ = T.ab3(op, q0, dt, n, hist=h)
    err_ab = np.sqrt(op.energy(q2 - eigenmode(M, n * dt))) / e0
    assert err_rk < 2e-4 and err_ab < 2 * err_rk


@pytest.mark.parametrize("N", [1, 2])
def test_eigenmode_h_convergence(N):
    # h^(N+1) on the 4^3 -> 8^3 pair (spatial error dominates: LSERK4 with a small dt);
    # the observed rate must be >= N + 0.7
    errs = []
    for n in (4, 8):
        mm = I.unit_cube_mesh(n)
        M = OMesh(get_ref(N), mm.verts, mm.etov, bc_default=BC_RIGID)
        op = Operator(M, np.ones(M.K), np.ones(M.K))
        T_end = 0.1
        steps = int(40 * n * (N + 1) ** 2 / 9) + 1
        q = T.lserk4(op, eigenmode(M, 0.0), T_end / steps, steps)
        errs.append(np.sqrt(op.energy(q - eigenmode(M, T_end)) / op.energy(eigenmode(M, 0.0))))
    rate = np.log2(errs[0] / errs[1])
    assert rate > N + 0.7, (errs, rate)


def test_lserk4_order_conditions():
    a, b, c = T.lserk4_coefficients()
    # convert 2N-storage form to Butcher form and check the order conditions up to order 4
    s = 5
    A = np.zeros((s, s))
    bb = np.zeros(s)
    # stage i uses res_i = a_i res_{i-1} + dt k_i; q += b_i res_i
    Bmat = np.zeros((s, s))                 # res_i = sum_j Bmat[i,j] k_j
    for i in range(s):
        if i > 0:
            Bmat[i] = a[i] * Bmat[i - 1]
        Bmat[i, i] += 1.0
    acc = np.zeros(s)
    for i in range(s):
        A[i] = acc.copy()                   # stage i evaluated at q after i updates
        acc = acc + b[i] * Bmat[i]
    bb = acc
    cc = A.sum(1)
    assert np.allclose(cc, c, atol=1e-12)
    conds = [bb.sum() - 1, bb @ cc - 1 / 2, bb @ cc ** 2 - 1 / 3, bb @ A @ cc - 1 / 6,
             bb @ cc ** 3 - 1 / 4, bb @ (cc * (A @ cc)) - 1 / 8, bb @ A @ cc ** 2 - 1 / 12, bb @ A @ A @ cc - 1 / 24]
    assert max(abs(x) for x in conds) < 1e-12


def test_levels_rules():
    m, op, lev, L, dtl = case("two_layer_small:6:6:4:3")
    M = op.m
    dt = local_dt(M.verts, M.etov, op.c, 3)
    assert L == 3 and dtl == dt.min()
    assert np.all(np.abs(lev[:, None] - lev[M.EToE]) <= 1)
    assert np.all(2.0 ** (L - lev) * dtl <= dt)
    # minimality: no element can be made coarser without violating a rule
    for k in np.nonzero(lev > 1)[0][:200]:
        l2 = lev[k] - 1
        ok_cfl = 2.0 ** (L - l2) * dtl <= dt[k]
        ok_nb = np.all(np.abs(l2 - lev[M.EToE[k]]) <= 1)
        assert not (ok_cfl and ok_nb)


def test_mrab_single_level_is_ab3_bitwise():
    m, op, lev, L, dtl = case("two_layer_small:4:4:3:2")
    rng = np.random.default_rng(5)
    q0 = rng.standard_normal((op.m.K, 4, op.ref.Np))
    st = T.MRAB(op, np.ones(op.m.K, dtype=int), 1, dtl)
    st.set_state(q0)
    for _ in range(6):
        st.global_step()
    q2, _ = T.ab3(op, q0, dtl, 6)
    assert np.array_equal(st.q, q2)
    # with a given history (r(-dt), r(-2 dt)): the first update uses r(0), r(-dt), r(-2 dt)
    h = rng.standard_normal((2, op.m.K, 4, op.ref.Np))
    st = T.MRAB(op, np.ones(op.m.K, dtype=int), 1, dtl)
    st.set_state(q0, hist2=h)
    st.global_step()
    q1, _ = T.ab3(op, q0, dtl, 1, hist=h)
    r0 = op.rhs(q0)
    assert np.array_equal(st.q, q1)
    assert np.allclose(q1, q0 + dtl * (23 / 12 * r0 - 16 / 12 * h[0] + 5 / 12 * h[1]), rtol=0, atol=1e-12)


def test_mrab_agrees_with_single_rate_to_third_order():
    # from rest with a source ~ t^3 (zero history is then exact); halving every step must
    # shrink the MRAB - single-rate difference by ~2^3
    m, op, lev, L, dtl = case("two_layer_small:4:4:3:2")
    assert L >= 2 and len(np.unique(lev)) >= 2
    M = op.m
    x = M.x
    g = np.exp(-((x[..., 0] - 1) ** 2 + (x[..., 1] - 1) ** 2 + (x[..., 2] - 0.5) ** 2) / 0.1)
    Tn = 32 * dtl

    def src_mr(r, t, ev):
        r[:, 0] += (t / Tn) ** 3 * g[ev]

    def src_sr(r, t):
        r[:, 0] += (t / Tn) ** 3 * g

    diffs = []
    for refine in (1, 2):
        d = dtl / refine
        st = T.MRAB(op, lev, L, d, src=src_mr)
        for _ in range(32 * refine):
            st.local_step()
        qs, _ = T.ab3(op, np.zeros_like(st.q), d, 32 * refine, src=src_sr)
        diffs.append(np.sqrt(op.energy(st.q - qs) / op.energy(qs)))
    assert diffs[0] / diffs[1] > 6.0, diffs


def test_neighbourhood_operator_gives_the_whole_mesh_rhs():
    """The sub-mesh oracle used for sampled checks on meshes too large to set up whole: at the
    sampled elements it reproduces the whole mesh's rhs (heterogeneous medium, mixed boundaries,
    both time directions)."""
    from tests.oracle_cases import neighbourhood_operator
    m, rho, c, N = I.config_mesh("two_layer_small:6:6:4:3")
    rng = np.random.default_rng(4)
    rho = rho * rng.uniform(0.8, 1.5, m.K)
    bc = rng.choice([BC_RIGID, BC_TRANSPARENT, BC_FREE], size=(m.K, 4))
    full = Operator(OMesh(get_ref(N), m.verts, m.etov, face_bc=bc), rho, c)
    el = np.sort(rng.choice(m.K, 60, replace=False))
    op, sub, loc = neighbourhood_operator(N, m.verts, m.etov, rho, c, el, face_bc=bc)
    assert sub.size < m.K and np.all(sub[loc] == el)
    q = rng.standard_normal((m.K, 4, full.ref.Np))
    for tau_sign in (1.0, -1.0):
        a = full.rhs(q, tau_sign=tau_sign, elems=el)
        b = op.rhs(q[sub], tau_sign=tau_sign, elems=loc)
        assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())
