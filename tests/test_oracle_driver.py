"""Algorithm 1 driver of the oracle on small seeded problems."""
import json
import os

import numpy as np

from qpat_inputs import make_problem, noise_draws
from qpat_inputs.configs import METHOD
from oracle import fem
from oracle.jacobian import Linearisation
from oracle.driver import reconstruct, initial_guess

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def simulate(P, g):
    lin = Linearisation(g, P.kappa, P.mu, P.phi_src)
    sig = P.cfg["noise"]
    xi = noise_draws(P.cfg["id"], P.n_ill, g.N)
    chi = lin.h + sig * np.abs(lin.h) * xi
    W = 1.0 / (sig * np.abs(lin.h))
    return chi, W, lin


def test_method_constants_match_paper():
    with open(os.path.join(GOLDEN, "method_constants.json")) as f:
        gold = json.load(f)
    for k in ("T", "delta", "b_over_a", "m0", "tau"):
        assert METHOD[k] == gold[k]


def test_initial_guess_homogeneous_data():
    """Noiseless data of the homogeneous medium gives mt_init = 0, kt_init = 0."""
    P = make_problem("T4", phantom="background")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    lin = Linearisation(g, np.full(g.N, P.kappa0), np.full(g.N, P.mu0), P.phi_src)
    beta = initial_guess(g, P.phi_src, lin.h, P.kappa0, P.mu0)
    assert np.abs(beta).max() < 1e-12


def test_reconstruction_reduces_nonlinear_residual():
    """The 16^3 face-source workload: residual falls towards sqrt(n_ill N), the
    whitened noise level (Sec. 4, remark after Algorithm 1)."""
    P = make_problem("C1")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    chi, W, _ = simulate(P, g)
    beta, log = reconstruct(g, P.phi_src, chi, W, P.kappa0, P.mu0, outer=2, inner=8)
    res = log["res_nl"]
    assert len(res) == 3
    assert res[1] < res[0] and res[2] < res[1]
    for hist in log["lsqr"]:
        assert np.all(np.diff(hist) <= 1e-12 * np.asarray(hist[:-1]))
    assert np.all(np.isfinite(beta))
    assert res[-1] < 0.25 * res[0]
    assert res[-1] > 0.9 * np.sqrt(P.n_ill * g.N)


def test_stop_on_reject_returns_previous_iterate():
    """Step 4: start at the true parameters; zero LSQR steps give beta = 0 (the
    homogeneous medium), whose residual is larger, so it is rejected and the
    previous beta is returned."""
    P = make_problem("T4")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    chi, W, _ = simulate(P, g)
    beta0 = np.concatenate([np.log(P.kappa / P.kappa0), np.log(P.mu / P.mu0)])
    beta, log = reconstruct(g, P.phi_src, chi, W, P.kappa0, P.mu0, outer=3, inner=0,
                            beta0=beta0, stop_on_reject=True)
    assert log["rejected"] == [True]
    assert np.array_equal(beta, beta0)


def test_fit_recovers_a_homogeneous_pair():
    """Noiseless data of a homogeneous medium (kappa*, mu*) other than the start:
    the background fit of the preamble returns (kappa*, mu*)."""
    from oracle.driver import fit_background
    P = make_problem("T4", phantom="background")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    ks, ms = 1.3 * P.kappa0, 0.8 * P.mu0
    h = Linearisation(g, np.full(g.N, ks), np.full(g.N, ms), P.phi_src).h
    k, m, it = fit_background(g, P.phi_src, h, 1.0 / np.abs(h), P.kappa0, P.mu0)
    assert abs(k / ks - 1) < 1e-9 and abs(m / ms - 1) < 1e-9, (k, m, it)
    assert 2 <= it < 30


def test_fit_matches_scipy_least_squares():
    """The fitted pair is the minimiser that a different method finds: SciPy's
    Levenberg-Marquardt on the same two-parameter residual, with a finite-difference
    Jacobian (no use of J)."""
    from scipy.optimize import least_squares
    from oracle.driver import fit_background
    P = make_problem("T4")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    chi, W, _ = simulate(P, g)
    k, m, _ = fit_background(g, P.phi_src, chi, W, P.kappa0, P.mu0)

    def resid(x):
        lin = Linearisation(g, np.full(g.N, np.exp(x[0])), np.full(g.N, np.exp(x[1])), P.phi_src)
        return (W * (chi - lin.h)).ravel()

    sol = least_squares(resid, np.log([P.kappa0, P.mu0]), method="lm", jac="2-point",
                        xtol=1e-15, ftol=1e-15, gtol=1e-15)
    assert abs(k / np.exp(sol.x[0]) - 1) < 1e-6 and abs(m / np.exp(sol.x[1]) - 1) < 1e-6, (k, m, sol.x)
    # the fit moved off the configured background: the data's mean level differs from it
    assert abs(m / P.mu0 - 1) > 1e-3


def test_step0_is_lsqr_on_the_kappa_block():
    """Step 0 of Sec. 5 on a 4^3 problem against textbook LSQR (SciPy) on the dense
    A L^{-1}, with A = W J_kt built column by column from J (brute force), L the
    Cholesky factor of M(kt_init) + delta I, the right-hand side
    W (chi - h + A kt_init) and the result mapped back by L^{-1}; mt is untouched."""
    from scipy.sparse.linalg import lsqr
    from oracle.driver import step0
    from oracle.jacobian import params
    from oracle import prior
    P = make_problem("T4")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    N = g.N
    chi, W, _ = simulate(P, g)
    beta = initial_guess(g, P.phi_src, chi, P.kappa0, P.mu0)
    beta[:N] = 0.05 * np.sin(np.arange(N))          # a non-zero kt_init
    lin = Linearisation(g, *params(P.kappa0, P.mu0, beta), P.phi_src)
    cols = []
    for j in range(N):
        e = np.zeros(2 * N)
        e[j] = 1.0
        cols.append((W * lin.jvp(e)).ravel())
    A = np.column_stack(cols)
    yt = (W * (chi - lin.h)).ravel() + A @ beta[:N]
    Mk = prior.M_of(g, beta[:N], METHOD["T"]).toarray() + METHOD["delta"] * np.eye(N)
    Linv = np.linalg.inv(np.linalg.cholesky(Mk).T)
    # a graded operator: plain LSQR (SciPy's, without reorthogonalisation) stays
    # accurate only for the first steps, as for the full problem
    for m in (1, 2):
        ref = Linv @ lsqr(A @ Linv, yt, atol=0, btol=0, conlim=0, iter_lim=m)[0]
        out, hist = step0(g, P.phi_src, chi, W, P.kappa0, P.mu0, beta, m, METHOD["T"], METHOD["delta"])
        assert np.linalg.norm(out[:N] - ref) <= 1e-9 * np.linalg.norm(ref), m
        assert np.array_equal(out[N:], beta[N:])
        assert abs(np.linalg.norm(A @ out[:N] - yt) - hist[-1]) <= 1e-9 * hist[-1]


def test_initial_guess_averages_exponentials_over_illuminations():
    """Sec. 4, paragraph after Algorithm 1: with several illuminations exp(mt_init)
    is the average over k of exp(mt_init^(k)) = chi_k / (mu0 phi0_k). Data
    chi_k = c_k mu0 phi0_k with distinct c_k give mt_init = log(mean_k c_k) at
    every node; a geometric mean (a mean of the logs) would give
    log(prod c_k)/4 = log(sqrt 2), far from log(1.875), and kt_init = 0."""
    P = make_problem("T4", n_ill=4)
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    lin0 = Linearisation(g, np.full(g.N, P.kappa0), np.full(g.N, P.mu0), P.phi_src)
    c = np.array([0.5, 1.0, 2.0, 4.0])
    chi = c[:, None] * P.mu0 * lin0.phi
    beta = initial_guess(g, P.phi_src, chi, P.kappa0, P.mu0)
    assert np.all(beta[:g.N] == 0.0)
    assert np.abs(beta[g.N:] - np.log(1.875)).max() <= 1e-14
    assert abs(np.log(1.875) - np.log(np.sqrt(2.0))) > 0.2


def test_discrepancy_principle_stops_below_the_noise_level():
    """Remark after Algorithm 1: stop PLSQR at the first step whose linearised
    residual is below sqrt(K N), the whitened noise level. On the 16^3 workload
    (data simulated on the reconstruction mesh, i.e. with the inverse crime) it
    fires in the third outer step; every history is a prefix of the fixed-count
    run's, ending at the first value under the level."""
    P = make_problem("C1")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    chi, W, _ = simulate(P, g)
    level = np.sqrt(chi.size)
    _, full = reconstruct(g, P.phi_src, chi, W, P.kappa0, P.mu0, outer=3, inner=30)
    _, dp = reconstruct(g, P.phi_src, chi, W, P.kappa0, P.mu0, outer=3, inner=30, discrepancy=1.0)
    assert dp["discrepancy_fired"] == [False, False, True]
    for h_full, h_dp in zip(full["lsqr"], dp["lsqr"]):
        m = len(h_dp) - 1
        np.testing.assert_allclose(h_dp, h_full[:m + 1], rtol=1e-12)
        below = [i for i in range(1, len(h_full)) if h_full[i] < level]
        if below:
            assert m == below[0] and h_dp[-1] < level <= h_dp[-2]
        else:
            assert m == 30
