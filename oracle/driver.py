"""Algorithm 1 (Sec. 4) with fixed outer / inner iteration counts -- oracle.

Test infrastructure only (see the package docstring).

Initialisation (Algorithm 1 preamble; several illuminations: Sec. 4, the
paragraph after the algorithm; Sec. 5 Test 1):
  kt_init = 0;  mu_init = mean_k chi_k / phi0_k with phi0_k the fluence of
  the homogeneous (kappa0, mu0);  mt_init = log(mu_init / mu0).
  (kappa0, mu0) are given, or fitted first (fit=True): the homogeneous pair
  minimising |W (chi - h(log(kappa) 1, log(mu) 1))| (Algorithm 1 preamble),
  by Gauss-Newton in (log kappa, log mu) -- the paper does not say how the
  minimiser is found; see fit_background.
Optional zeroth step (Sec. 5, step0_inner > 0): PLSQR for kt alone with the
  Jacobian's kt columns and M(kt_init) + delta I, from kt = 0, with the
  right-hand side W (chi - h + J_kt kt_init); its solution replaces kt_init.
Each outer step l:
  1. h = h(beta_l), yt = W (chi - h + J beta_l)         (W = Gamma^{-1/2}, diagonal)
  2. M_delta from kt_l, mt_l
  3. PLSQR on A = W J from 0 -> beta_{l+1}; a fixed count, the window rule
     r_m <= tau (eq. (4.11)) and/or the discrepancy principle of the remark
     after Algorithm 1 (stop once the linearised residual is below
     fudge * sqrt(n_ill N), the whitened noise level; option `discrepancy`)
  4. nonlinear residual ||W (chi - h(beta_{l+1}))|| compared with ||W (chi - h)||;
     with stop_on_reject the previous iterate is returned when it did not
     decrease, otherwise the comparison is only recorded.
"""
import numpy as np

import scipy.sparse as sp

from .jacobian import Linearisation, params
from .prior import Prior, M_of, DeflatedDirect
from .plsqr import plsqr
from .solve import make_solver


def background_misfit(geo, phi_src, chi, W, kappa, mu, solver="direct", rtol=1e-10):
    """|W (chi - h(kappa 1, mu 1))|^2 and the homogeneous linearisation."""
    lin = Linearisation(geo, np.full(geo.N, kappa), np.full(geo.N, mu), phi_src, solver, rtol)
    return float(np.sum((W * (chi - lin.h)) ** 2)), lin


def fit_background(geo, phi_src, chi, W, kappa_start, mu_start, maxit=30, tol=1e-10,
                   solver="direct", rtol=1e-10):
    """Gauss-Newton for (a, b) = (log kappa, log mu) minimising
    F = |W (chi - h(e^a 1, e^b 1))|^2. The columns of the 2-parameter Jacobian
    are J [1; 0] and J [0; 1] (derivatives in the log-parameters, Appendix);
    the step solves the linear least-squares problem min |C d - r| with
    C = [W J[1;0], W J[0;1]], r = W (chi - h). A step longer than 1 in either
    log is shortened to 1, then halved (at most 30 times) until F does not
    increase. Stops when the accepted step is <= tol in both logs, when no
    halving decreases F, or after maxit steps. Returns (kappa0, mu0, iters)."""
    chi = np.asarray(chi)
    W = np.asarray(W)
    N = geo.N
    a, b = np.log(kappa_start), np.log(mu_start)
    F, lin = background_misfit(geo, phi_src, chi, W, np.exp(a), np.exp(b), solver, rtol)
    one, zero = np.ones(N), np.zeros(N)
    it = 0
    while it < maxit:
        c1 = (W * lin.jvp(np.concatenate([one, zero]))).ravel()
        c2 = (W * lin.jvp(np.concatenate([zero, one]))).ravel()
        r = (W * (chi - lin.h)).ravel()
        d = np.linalg.lstsq(np.column_stack([c1, c2]), r, rcond=None)[0]
        d = d / max(1.0, np.abs(d).max())
        t = 1.0
        for _ in range(31):
            Fn, lin_n = background_misfit(geo, phi_src, chi, W, np.exp(a + t * d[0]), np.exp(b + t * d[1]),
                                          solver, rtol)
            if Fn <= F:
                break
            t *= 0.5
        else:
            break
        a, b, F, lin = a + t * d[0], b + t * d[1], Fn, lin_n
        it += 1
        if np.abs(t * d).max() <= tol:
            break
    return float(np.exp(a)), float(np.exp(b)), it


def step0(geo, phi_src, chi, W, kappa0, mu0, beta_init, inner, T=5e-3, delta=1e-6,
          solver="direct", rtol=1e-10, m0=None, tau=None, prior="pm", q=1.0, prior_solver=None):
    """Zeroth step of Sec. 5: PLSQR on A = W J_kt (the kt columns of J at
    beta_init) with prior M(kt_init) + delta I (N x N), right-hand side
    W (chi - h + J_kt kt_init), from 0. Returns (beta with kt replaced, history)."""
    chi = np.asarray(chi)
    W = np.asarray(W)
    N = geo.N
    kappa, mu = params(kappa0, mu0, beta_init)
    lin = Linearisation(geo, kappa, mu, phi_src, solver, rtol)
    zero = np.zeros(N)
    kt = np.asarray(beta_init[:N])
    yt = (W * (chi - lin.h + lin.jvp(np.concatenate([kt, zero])))).ravel()
    Mk = (M_of(geo, kt, T, prior, q) + delta * sp.identity(N)).tocsr()
    n_ill = lin.n_ill

    def A(v):
        return (W * lin.jvp(np.concatenate([v, zero]))).ravel()

    def At(u):
        return lin.vjp(W * u.reshape(n_ill, N))[:N]

    ps = prior_solver or solver
    Minv = DeflatedDirect(Mk, N, delta) if ps == "deflated" else make_solver(Mk, ps, rtol)
    it = plsqr(A, At, Minv, yt, inner, m0, tau)
    return np.concatenate([it.x, np.asarray(beta_init[N:])]), list(it.history)


def initial_guess(geo, phi_src, chi, kappa0, mu0, solver="direct", rtol=1e-10):
    N = geo.N
    lin0 = Linearisation(geo, np.full(N, kappa0), np.full(N, mu0), phi_src, solver, rtol)
    ratio = np.mean(np.asarray(chi) / lin0.phi, axis=0)
    mu_init = np.maximum(ratio, 1e-12 * mu0)
    return np.concatenate([np.zeros(N), np.log(mu_init / mu0)])


def reconstruct(geo, phi_src, chi, W, kappa0, mu0, outer, inner, T=5e-3,
                b_over_a=1.0, delta=1e-6, solver="direct", rtol=1e-10,
                beta0=None, stop_on_reject=False, m0=None, tau=None, prior="pm", q=1.0,
                fit=False, step0_inner=0, discrepancy=None, prior_solver=None):
    """discrepancy: None, or the factor of the noise level sqrt(n_ill N) at
    which step 3 stops (1.0: the plain discrepancy principle); log["discrepancy_fired"]
    records per outer step whether it ended the LSQR run. prior_solver: how
    M_delta^{-1} is applied ("direct", "pcg" or "deflated"; default: solver)."""
    ps = prior_solver or solver
    chi = np.asarray(chi)
    W = np.asarray(W)
    N = geo.N
    log = dict(res_nl=[], lsqr=[], rejected=[], discrepancy_fired=[])
    level = None if discrepancy is None else float(discrepancy) * np.sqrt(chi.size)
    if fit:
        kappa0, mu0, log["fit_iters"] = fit_background(geo, phi_src, chi, W, kappa0, mu0, solver=solver, rtol=rtol)
    log["kappa0"], log["mu0"] = kappa0, mu0
    beta = initial_guess(geo, phi_src, chi, kappa0, mu0, solver, rtol) if beta0 is None \
        else np.array(beta0, dtype=np.float64)
    if step0_inner > 0:
        beta, log["step0"] = step0(geo, phi_src, chi, W, kappa0, mu0, beta, step0_inner, T, delta, solver, rtol,
                                   m0, tau, prior, q, prior_solver=ps)
    lin = None
    for l in range(outer):
        kappa, mu = params(kappa0, mu0, beta)
        lin = Linearisation(geo, kappa, mu, phi_src, solver, rtol) if lin is None else lin
        res = np.linalg.norm(W * (chi - lin.h))
        log["res_nl"].append(res)
        yt = (W * (chi - lin.h + lin.jvp(beta))).ravel()
        Md = Prior(geo, beta[:N], beta[N:], T, b_over_a, delta, ps, rtol, kind=prior, q=q)
        n_ill = lin.n_ill

        def A(v, lin=lin):
            return (W * lin.jvp(v)).ravel()

        def At(u, lin=lin):
            return lin.vjp(W * u.reshape(n_ill, N))

        it = plsqr(A, At, Md.solve, yt, inner, m0, tau, noise_level=level)
        log["lsqr"].append(list(it.history))
        log["discrepancy_fired"].append(level is not None and it.history[-1] < level)
        beta_new = it.x
        kappa_n, mu_n = params(kappa0, mu0, beta_new)
        lin_new = Linearisation(geo, kappa_n, mu_n, phi_src, solver, rtol)
        res_new = np.linalg.norm(W * (chi - lin_new.h))
        rejected = res_new >= res
        log["rejected"].append(bool(rejected))
        if rejected and stop_on_reject:
            log["res_nl"].append(res)
            return beta, log
        beta, lin = beta_new, lin_new
    log["res_nl"].append(np.linalg.norm(W * (chi - lin.h)) if lin is not None else None)
    return beta, log


def finer_mesh_data(geo_fine, kappa_fine, mu_fine, phi_src_fine, inj, solver="direct", rtol=1e-10):
    """Noiseless data without the obvious inverse crime (Sec. 2, the footnote on
    the measurement model; Sec. 5): H = mu phi computed with P1 elements on a
    denser mesh, then its nodal values at the reconstruction mesh's nodes. On
    nested Kuhn meshes every coarse node is a fine node, so interpolation is the
    index map inj. Returns [n_ill][N_coarse]."""
    lin = Linearisation(geo_fine, kappa_fine, mu_fine, phi_src_fine, solver, rtol)
    return lin.h[:, inj]
