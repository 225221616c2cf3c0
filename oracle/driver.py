"""Algorithm 1 (Sec. 4) with fixed outer / inner iteration counts -- oracle.

Test infrastructure only (see the package docstring).

Initialisation (Algorithm 1 preamble; several illuminations: Sec. 4, the
paragraph after the algorithm; Sec. 5 Test 1):
  kt_init = 0;  mu_init = mean_k chi_k / phi0_k with phi0_k the fluence of
  the homogeneous (kappa0, mu0);  mt_init = log(mu_init / mu0).
  (kappa0, mu0) are given (the background fit of the preamble is not done).
Each outer step l:
  1. h = h(beta_l), yt = W (chi - h + J beta_l)         (W = Gamma^{-1/2}, diagonal)
  2. M_delta from kt_l, mt_l
  3. PLSQR on A = W J from 0 -> beta_{l+1}
  4. nonlinear residual ||W (chi - h(beta_{l+1}))|| compared with ||W (chi - h)||;
     with stop_on_reject the previous iterate is returned when it did not
     decrease, otherwise the comparison is only recorded.
"""
import numpy as np

from .jacobian import Linearisation, params
from .prior import Prior
from .plsqr import plsqr


def initial_guess(geo, phi_src, chi, kappa0, mu0, solver="direct", rtol=1e-10):
    N = geo.N
    lin0 = Linearisation(geo, np.full(N, kappa0), np.full(N, mu0), phi_src, solver, rtol)
    ratio = np.mean(np.asarray(chi) / lin0.phi, axis=0)
    mu_init = np.maximum(ratio, 1e-12 * mu0)
    return np.concatenate([np.zeros(N), np.log(mu_init / mu0)])


def reconstruct(geo, phi_src, chi, W, kappa0, mu0, outer, inner, T=5e-3,
                b_over_a=1.0, delta=1e-6, solver="direct", rtol=1e-10,
                beta0=None, stop_on_reject=False, m0=None, tau=None, prior="pm", q=1.0):
    chi = np.asarray(chi)
    W = np.asarray(W)
    N = geo.N
    beta = initial_guess(geo, phi_src, chi, kappa0, mu0, solver, rtol) if beta0 is None \
        else np.array(beta0, dtype=np.float64)
    log = dict(res_nl=[], lsqr=[], rejected=[])
    lin = None
    for l in range(outer):
        kappa, mu = params(kappa0, mu0, beta)
        lin = Linearisation(geo, kappa, mu, phi_src, solver, rtol) if lin is None else lin
        res = np.linalg.norm(W * (chi - lin.h))
        log["res_nl"].append(res)
        yt = (W * (chi - lin.h + lin.jvp(beta))).ravel()
        Md = Prior(geo, beta[:N], beta[N:], T, b_over_a, delta, solver, rtol, kind=prior, q=q)
        n_ill = lin.n_ill

        def A(v, lin=lin):
            return (W * lin.jvp(v)).ravel()

        def At(u, lin=lin):
            return lin.vjp(W * u.reshape(n_ill, N))

        it = plsqr(A, At, Md.solve, yt, inner, m0, tau)
        log["lsqr"].append(list(it.history))
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
