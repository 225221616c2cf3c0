"""Pins of the oracle's FEM (assembly, load vector, forward solve).

Each check compares against something other than the oracle's own formula:
textbook integrals, exact solutions of the PDE, conservation, invariants.
"""
import itertools
from math import factorial

import numpy as np
import pytest

from qpat_inputs import kuhn_mesh, make_problem
from oracle import fem
from oracle.solve import Direct, pcg

L = 40.0
NORMALS = np.array([[0, 0, -1], [0, 0, 1], [-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0]], float)


def geo_of(m):
    return fem.geometry(m.coords, m.tets, m.bfaces)


def test_tet_quadrature_is_exact_to_degree_3():
    """int_T lambda^alpha = 6|T| alpha! / (|alpha| + 3)! (Dirichlet integral)."""
    for alpha in itertools.product(range(4), repeat=4):
        if sum(alpha) > 3:
            continue
        exact = 6.0 * np.prod([factorial(a) for a in alpha]) / factorial(sum(alpha) + 3)
        quad = np.sum(fem._TET_W * np.prod(fem._TET_PTS ** np.array(alpha), axis=1))
        assert abs(quad - exact) < 1e-15, alpha


def test_tri_quadrature_is_exact_to_degree_2():
    for alpha in itertools.product(range(3), repeat=3):
        if sum(alpha) > 2:
            continue
        exact = 2.0 * np.prod([factorial(a) for a in alpha]) / factorial(sum(alpha) + 2)
        quad = np.sum(fem._TRI_W * np.prod(fem._TRI_PTS ** np.array(alpha), axis=1))
        assert abs(quad - exact) < 1e-15, alpha


def test_geometry_gradients_and_measures():
    rng = np.random.default_rng(0)
    coords = rng.standard_normal((4, 3))
    geo = fem.geometry(coords, np.array([[0, 1, 2, 3]]), np.array([[0, 1, 2]]))
    # grad(lambda_a) . (x_b - x_0) = delta_ab - delta_a0
    for a in range(4):
        for b in range(4):
            want = (a == b) - (a == 0)
            assert abs(geo.grad[0, a] @ (coords[b] - coords[0]) - want) < 1e-12
    m = kuhn_mesh(4, L)
    g = geo_of(m)
    assert np.isclose(g.vol.sum(), L ** 3, rtol=1e-13)
    assert np.isclose(g.area.sum(), 6 * L ** 2, rtol=1e-13)


def test_assembly_invariants():
    P = make_problem("T8")
    g = geo_of(P.mesh)
    N = g.N
    one = np.ones(N)
    S = fem.stiffness(g, P.kappa)
    assert np.abs(S @ one).max() < 1e-12 * np.abs(S).max()
    K = fem.system_matrix(g, P.kappa, P.mu)
    assert abs(K - K.T).max() <= 1e-15 * abs(K).max()
    B = fem.boundary_mass(g)
    assert np.isclose(one @ (B @ one), 6 * L ** 2, rtol=1e-13)
    Mm = fem.mass(g, P.mu)
    want = np.sum(g.vol * P.mu[g.tets].mean(axis=1))
    assert np.isclose(one @ (Mm @ one), want, rtol=1e-13)


def test_constant_coefficient_mass_is_textbook():
    """Constant mu: element mass mu |T| (1 + delta_ab) / 20."""
    m = kuhn_mesh(1, L)
    g = geo_of(m)
    M = fem.mass(g, np.full(m.N, 0.7)).toarray()
    want = np.zeros_like(M)
    for e, t in enumerate(m.tets):
        for a in range(4):
            for b in range(4):
                want[t[a], t[b]] += 0.7 * g.vol[e] * (1 + (a == b)) / 20.0
    assert np.allclose(M, want, rtol=1e-13, atol=0)


def test_load_vector_unit_face_source():
    """A unit source on one face: sum_i f_i = 2 L^2 (Appendix weak form: 2 int Phi v)."""
    m = kuhn_mesh(5, L)
    g = geo_of(m)
    src = np.zeros((1, m.F_b, 3))
    src[0, m.bface_tag == 2] = 1.0
    f = fem.load_vectors(g, src)[0]
    assert np.isclose(f.sum(), 2 * L ** 2, rtol=1e-13)
    assert np.all(f[np.abs(m.coords[:, 0]) > 1e-9] == 0.0)


def patch_problem(n, kap, a, b):
    m = kuhn_mesh(n, L)
    g = geo_of(m)
    K = fem.system_matrix(g, np.full(m.N, kap), np.zeros(m.N))
    phis = a + m.coords @ b
    nu = NORMALS[m.bface_tag]
    src = 0.25 * phis[m.bfaces] + 0.5 * kap * (nu @ b)[:, None]
    f = fem.load_vectors(g, src[None])[0]
    return m, K, f, phis


def test_patch_test_linear_solution_is_exact():
    """mu = 0, constant kappa: phi* = a + b.x solves eq. (2.1) with
    Phi = phi*/4 + (kappa/2) b.nu, linear on each boundary face, so P1 is exact."""
    m, K, f, phis = patch_problem(4, 0.37, 2.0, np.array([0.01, -0.02, 0.015]))
    x = Direct(K)(f)
    assert np.abs(x - phis).max() < 1e-12


def homogeneous_error(n, kap=1 / 3.03, mu=0.01):
    """phi*(x) = exp(-k x), k = sqrt(mu/kappa), solves -kappa phi'' + mu phi = 0;
    Robin data Phi = phi*/4 + (kappa/2) d(phi*)/d(nu) on each face."""
    m = kuhn_mesh(n, L)
    g = geo_of(m)
    k = np.sqrt(mu / kap)
    K = fem.system_matrix(g, np.full(m.N, kap), np.full(m.N, mu))
    pts = m.coords[m.bfaces]
    e = np.exp(-k * pts[..., 0])
    dn = -k * e * NORMALS[m.bface_tag][:, None, 0]
    f = fem.load_vectors(g, (0.25 * e + 0.5 * kap * dn)[None])[0]
    x = pcg(K, f, rtol=1e-13)
    err = x - np.exp(-k * m.coords[:, 0])
    X = m.coords
    inner = np.all((X > 1e-9) & (X < L - 1e-9), axis=1)
    return np.sqrt(np.mean(err ** 2)), np.abs(err[inner]).max()


def test_homogeneous_closed_form_second_order():
    e8, i8 = homogeneous_error(8)
    e16, i16 = homogeneous_error(16)
    e32, i32 = homogeneous_error(32)
    assert 3.5 < e8 / e16 < 4.6 and 3.5 < e16 / e32 < 4.6
    assert 3.5 < i8 / i16 < 4.6 and 3.5 < i16 / i32 < 4.6
    assert e32 < 1e-3


def test_conservation():
    """int mu_h phi_h dx + 1/2 int_bdry phi_h dS = 2 int_bdry Phi_h dS."""
    P = make_problem("T8")
    g = geo_of(P.mesh)
    K = fem.system_matrix(g, P.kappa, P.mu)
    f = fem.load_vectors(g, P.phi_src)
    phi = Direct(K)(f)
    for k in range(P.n_ill):
        mu_q = P.mu[g.tets] @ fem._TET_PTS.T
        ph_q = phi[k][g.tets] @ fem._TET_PTS.T
        vol_int = np.sum(g.vol * ((mu_q * ph_q) @ fem._TET_W))
        bq = phi[k][g.bfaces] @ fem._TRI_PTS.T
        bdry_int = np.sum(g.area * (bq @ fem._TRI_W))
        src_q = P.phi_src[k] @ fem._TRI_PTS.T
        src_int = np.sum(g.area * (src_q @ fem._TRI_W))
        lhs = vol_int + 0.5 * bdry_int
        assert abs(lhs - 2 * src_int) < 1e-12 * abs(2 * src_int)


def test_direct_and_pcg_agree():
    P = make_problem("T12")
    g = geo_of(P.mesh)
    K = fem.system_matrix(g, P.kappa, P.mu)
    f = fem.load_vectors(g, P.phi_src)
    xd = Direct(K)(f)
    info = {}
    xc = pcg(K, f[0], rtol=1e-14, info=info)
    assert info["relres"] <= 1e-14
    assert np.linalg.norm(xc - xd[0]) <= 1e-12 * np.linalg.norm(xd[0])


def test_load_matrices_match_coefficient_derivatives():
    """K is linear in the nodal coefficients, so dK/dkappa_j phi = S(e_j) phi and
    dK/dmu_j phi = Mass(e_j) phi; G(1) and G(2) must be minus those columns
    (Appendix, definition of G)."""
    m = kuhn_mesh(2, L)
    g = geo_of(m)
    rng = np.random.default_rng(3)
    phi = rng.uniform(0.5, 1.5, m.N)
    G1 = fem.load_matrix_G1(g, phi).toarray()
    G2 = fem.load_matrix_G2(g, phi).toarray()
    for j in range(m.N):
        e = np.zeros(m.N)
        e[j] = 1.0
        assert np.allclose(G1[:, j], -(fem.stiffness(g, e) @ phi), atol=1e-13)
        assert np.allclose(G2[:, j], -(fem.mass(g, e) @ phi), atol=1e-13)
    assert np.allclose(G2, G2.T, atol=1e-15)


def test_finer_mesh_data_is_the_fine_solution_at_coarse_nodes():
    """Data without the obvious inverse crime (simulated on the 2n mesh, read at the
    coarse nodes) for the closed form exp(-kx): it carries the fine mesh's O((h/2)^2)
    nodal error, a quarter of the coarse mesh's own. A wrong node map would leave an
    O(1) error."""
    from qpat_inputs import coarse_in_fine
    from oracle.jacobian import Linearisation
    from oracle.driver import finer_mesh_data
    kap, mu, n = 1 / 3.03, 0.01, 8
    k = np.sqrt(mu / kap)

    def robin(m):
        pts = m.coords[m.bfaces]
        e = np.exp(-k * pts[..., 0])
        return (0.25 * e + 0.5 * kap * (-k * e * NORMALS[m.bface_tag][:, None, 0]))[None]

    mc, mf = kuhn_mesh(n, L), kuhn_mesh(2 * n, L)
    gc, gf = geo_of(mc), geo_of(mf)
    hc = Linearisation(gc, np.full(mc.N, kap), np.full(mc.N, mu), robin(mc)).h[0]
    hf = finer_mesh_data(gf, np.full(mf.N, kap), np.full(mf.N, mu), robin(mf), coarse_in_fine(n))[0]
    exact = mu * np.exp(-k * mc.coords[:, 0])
    ec = np.sqrt(np.mean((hc - exact) ** 2))
    ef = np.sqrt(np.mean((hf - exact) ** 2))
    assert 3.5 < ec / ef < 4.6, (ec, ef)
    assert np.abs(hf - exact).max() < 1e-2 * np.abs(exact).max()
