"""Pins of the oracle's J s and J^T t (Appendix formulas)."""
import numpy as np
import pytest

from qpat_inputs import kuhn_mesh, make_problem, gaussian_sources, probe_vectors
from oracle import fem
from oracle.jacobian import Linearisation, params
from oracle.solve import Direct


def small_problem(n=2, n_ill=2, seed=7):
    m = kuhn_mesh(n, 40.0)
    g = fem.geometry(m.coords, m.tets, m.bfaces)
    rng = np.random.default_rng(seed)
    beta = 0.3 * rng.standard_normal(2 * m.N)
    src = gaussian_sources(m, n_ill, sigma=15.0)
    return m, g, beta, src


def h_of(g, beta, src, k0=0.33, m0=0.01):
    kappa, mu = params(k0, m0, beta)
    return Linearisation(g, kappa, mu, src).h


def test_central_differences():
    """||J s - (h(b + e s) - h(b - e s)) / 2e|| / ||J s|| small, and O(e^2)."""
    m, g, beta, src = small_problem(3, 2)
    kappa, mu = params(0.33, 0.01, beta)
    lin = Linearisation(g, kappa, mu, src)
    rng = np.random.default_rng(1)
    s = rng.standard_normal(2 * m.N)
    Js = lin.jvp(s)
    errs = []
    for eps in (1e-3, 5e-4):
        fd = (h_of(g, beta + eps * s, src) - h_of(g, beta - eps * s, src)) / (2 * eps)
        errs.append(np.linalg.norm(Js - fd) / np.linalg.norm(Js))
    assert errs[0] < 1e-5
    assert 3.0 < errs[0] / errs[1] < 5.0        # second-order in eps
    eps = 1e-5
    fd = (h_of(g, beta + eps * s, src) - h_of(g, beta - eps * s, src)) / (2 * eps)
    assert np.linalg.norm(Js - fd) / np.linalg.norm(Js) < 1e-8


def test_adjoint_identity():
    """<J s, t> = <s, J^T t> with direct solves."""
    P = make_problem("T8")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    lin = Linearisation(g, P.kappa, P.mu, P.phi_src)
    s, t = probe_vectors(P.cfg["id"], P.n_ill, g.N)
    lhs = np.sum(lin.jvp(s) * t)
    rhs = s @ lin.vjp(t)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def test_dense_jacobian_by_direct_differentiation():
    """On a 2^3 mesh, build dh/dbeta without G: h = mu * K^{-1} f, K linear in the
    nodal coefficients, so dh/dkt_j = -mu K^{-1} S(kappa_j e_j) phi and
    dh/dmt_j = -mu K^{-1} Mass(mu_j e_j) phi + mu_j phi_j e_j."""
    m, g, beta, src = small_problem(2, 2)
    kappa, mu = params(0.33, 0.01, beta)
    lin = Linearisation(g, kappa, mu, src)
    N = m.N
    K = fem.system_matrix(g, kappa, mu)
    solve = Direct(K)
    J = lin.dense_jacobian()
    Jref = np.zeros_like(J)
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        for k in range(2):
            rows = slice(k * N, (k + 1) * N)
            dphi_k = -solve(fem.stiffness(g, kappa[j] * e) @ lin.phi[k])
            dphi_m = -solve(fem.mass(g, mu[j] * e) @ lin.phi[k])
            Jref[rows, j] = mu * dphi_k
            Jref[rows, N + j] = mu * dphi_m + mu[j] * lin.phi[k][j] * e
    assert np.abs(J - Jref).max() <= 1e-12 * np.abs(Jref).max()
    # and the transpose product is the dense transpose
    rng = np.random.default_rng(2)
    t = rng.standard_normal((2, N))
    assert np.allclose(lin.vjp(t), J.T @ t.ravel(), rtol=1e-11, atol=1e-14 * np.abs(J).max())


def test_jvp_is_linear():
    P = make_problem("T4")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    lin = Linearisation(g, P.kappa, P.mu, P.phi_src)
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal((2, 2 * g.N))
    lhs = lin.jvp(2.0 * a - 3.0 * b)
    rhs = 2.0 * lin.jvp(a) - 3.0 * lin.jvp(b)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-14 * np.abs(rhs).max())
