"""Pins of the oracle's priorconditioned LSQR against SciPy's LSQR and dense algebra."""
import numpy as np
import pytest
from scipy.sparse.linalg import lsqr

from qpat_inputs import make_problem, probe_vectors
from oracle import fem, prior
from oracle.jacobian import Linearisation
from oracle.plsqr import PLSQR, plsqr, window_ratio


def scipy_lsqr(A, b, m):
    return lsqr(A, b, damp=0.0, atol=0.0, btol=0.0, conlim=0.0, iter_lim=m)[0]


def random_spd(n, rng):
    Q = rng.standard_normal((n, n))
    return Q @ Q.T + 0.5 * np.eye(n)


@pytest.mark.parametrize("m", [1, 2, 5, 9])
def test_identity_prior_is_textbook_lsqr(m):
    rng = np.random.default_rng(m)
    A = rng.standard_normal((30, 12))
    b = rng.standard_normal(30)
    ref = scipy_lsqr(A, b, m)
    for reorth in (False, True):
        it = plsqr(lambda v: A @ v, lambda u: A.T @ u, lambda p: p.copy(), b, m, reorth=reorth)
        assert np.linalg.norm(it.x - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("m", [1, 3, 7])
def test_priorconditioned_equals_lsqr_on_A_Linv(m):
    """M = L^T L: PLSQR(A, M) = L^{-1} LSQR(A L^{-1}, b) (Sec. 4, eq. (4.10))."""
    rng = np.random.default_rng(10 + m)
    A = rng.standard_normal((25, 10))
    b = rng.standard_normal(25)
    M = random_spd(10, rng)
    C = np.linalg.cholesky(M)          # M = C C^T, so L = C^T
    Lmat = C.T
    Linv = np.linalg.inv(Lmat)
    ref = Linv @ scipy_lsqr(A @ Linv, b, m)
    for reorth in (False, True):
        it = plsqr(lambda v: A @ v, lambda u: A.T @ u, lambda p: np.linalg.solve(M, p), b, m,
                   reorth=reorth)
        assert np.linalg.norm(it.x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_residual_estimate_and_full_krylov():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((20, 8))
    b = rng.standard_normal(20)
    M = random_spd(8, rng)
    it = PLSQR(lambda v: A @ v, lambda u: A.T @ u, lambda p: np.linalg.solve(M, p), b)
    prev = np.inf
    for _ in range(8):
        est = it.step()
        true = np.linalg.norm(A @ it.x - b)
        assert abs(est - true) <= 1e-10 * true
        assert est <= prev * (1 + 1e-14)
        prev = est
    # after n steps: the least-squares solution of the full-rank tall system
    xls = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(it.x - xls) <= 1e-9 * np.linalg.norm(xls)


def test_iterates_lie_in_range_of_Minv():
    """x_m = M^{-1} z with z in the Krylov space span{(A^T A M^{-1})^j A^T b}."""
    rng = np.random.default_rng(6)
    A = rng.standard_normal((30, 15))
    b = rng.standard_normal(30)
    M = random_spd(15, rng)
    Minv = np.linalg.inv(M)
    m = 4
    it = plsqr(lambda v: A @ v, lambda u: A.T @ u, lambda p: Minv @ p, b, m)
    basis = [A.T @ b]
    for _ in range(m - 1):
        basis.append(A.T @ (A @ (Minv @ basis[-1])))
    B = np.stack(basis, axis=1)
    z = M @ it.x
    coef = np.linalg.lstsq(B, z, rcond=None)[0]
    assert np.linalg.norm(B @ coef - z) <= 1e-8 * np.linalg.norm(z)


def test_plsqr_on_the_qpat_operator_matches_scipy():
    """A = W J of a 4^3 problem, M_delta of its log-parameters, against dense LSQR."""
    P = make_problem("T4")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    lin = Linearisation(g, P.kappa, P.mu, P.phi_src)
    N, n_ill = g.N, P.n_ill
    W = 1.0 / (0.01 * np.abs(lin.h))
    J = lin.dense_jacobian()
    A = W.ravel()[:, None] * J
    kt, mt = np.log(P.kappa / P.kappa0), np.log(P.mu / P.mu0)
    Md = prior.M_delta(g, kt, mt).toarray()
    s, t = probe_vectors(P.cfg["id"], n_ill, N)
    yt = t.ravel()
    C = np.linalg.cholesky(Md)
    Linv = np.linalg.inv(C.T)
    Aop = lambda v: (W * lin.jvp(v)).ravel()
    Atop = lambda u: lin.vjp(W * u.reshape(n_ill, N))
    # a graded operator: plain LSQR stays accurate only for the first steps
    for m in (1, 2):
        ref = Linv @ scipy_lsqr(A @ Linv, yt, m)
        for reorth in (False, True):
            it = plsqr(Aop, Atop, lambda p: np.linalg.solve(Md, p), yt, m, reorth=reorth)
            assert np.linalg.norm(it.x - ref) <= 1e-9 * np.linalg.norm(ref)
    # with reorthogonalisation the residual history is reproducible and the
    # iterate stable under a 1e-12 relative perturbation of M_delta^{-1}
    a = plsqr(Aop, Atop, lambda p: np.linalg.solve(Md, p), yt, 12)
    wig = 1.0 + 1e-12 * np.sin(np.arange(2 * N))
    b = plsqr(Aop, Atop, lambda p: np.linalg.solve(Md, p) * wig, yt, 12)
    ha, hb = np.array(a.history), np.array(b.history)
    assert np.all(np.abs(ha - hb) <= 1e-11 * ha)
    assert np.all(np.diff(ha) <= 1e-12 * ha[:-1])
    assert np.linalg.norm(a.x - b.x) <= 1e-5 * np.linalg.norm(a.x)
    # and the residual estimate is the true residual
    assert abs(np.linalg.norm(A @ a.x - yt) - ha[-1]) <= 1e-9 * ha[-1]


def test_zero_rhs_returns_zero():
    A = np.eye(3)
    it = plsqr(lambda v: A @ v, lambda u: A.T @ u, lambda p: p, np.zeros(3), 3)
    assert np.all(it.x == 0.0)


def test_window_ratio():
    hist = [10.0, 9.0, 8.0, 7.0]
    assert window_ratio(hist, 2, 2) is None
    assert np.isclose(window_ratio(hist, 3, 2), 1 - 7.0 / 9.0)
