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
