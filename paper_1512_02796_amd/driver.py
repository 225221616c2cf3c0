"""Algorithm 1 (Sec. 4) on the GPU library, with fixed or adaptive counts.

Host control flow only: every vector operation is a libqpat call (forward
solve, misfit, initial guess, prior assembly, LSQR). The host sees scalars
(residual norms) and decides what to call next.

  fit   : optionally the homogeneous (kappa0, mu0) minimising |W (chi - h)|
          (preamble; qpat_fit_background)
  init  : kt = 0, mt = log(mean_k chi_k / phi0_k / mu0), phi0 the fluence of
          the homogeneous (kappa0, mu0) (preamble; several illuminations:
          paragraph after Algorithm 1 and Sec. 5)
  step 0: optionally PLSQR for kt alone with M(kt_init) + delta I (Sec. 5;
          qpat_lsqr_init_kappa); its solution replaces kt_init
  step 1: h = h(beta_l); yt = W (chi - h + J beta_l)     (inside qpat_lsqr_init)
  step 2: M_delta from kt_l, mt_l                          (qpat_prior_setup)
  step 3: PLSQR from 0: `inner` steps, or until r_m <= tau over a window of
          m0 steps (eq. (4.11)) when m0 and tau are given, or -- with
          `discrepancy` -- until the residual of the linearised model is below
          discrepancy * sqrt(n_ill N), the whitened noise level (Morozov's
          discrepancy principle, the remark after Algorithm 1)
  step 4: if ||W (chi - h(beta_{l+1}))|| >= ||W (chi - h(beta_l))|| the step
          is rejected; with stop_on_reject the previous iterate is returned,
          otherwise the comparison is only recorded.
"""
import math

import torch


def window_ratio(history, m, m0):
    """r_m = 1 - res_m / res_{m-m0} for m > m0 (eq. (4.11)); history[0] = res_0."""
    if m <= m0:
        return None
    den = history[m - m0]
    return 1.0 - history[m] / den if den > 0 else 0.0


def reconstruct(ctx, chi, W, kappa0, mu0, outer, inner, T=5e-3, b_over_a=1.0, delta=1e-6,
                beta0=None, stop_on_reject=False, m0=None, tau=None, prior="pm", q=1.0,
                fit=False, step0_inner=0, discrepancy=None):
    """prior: "pm" (Perona-Malik) or "tvq" (r(t) = T^(2-q) (t^2 + T^2)^(q/2) / q).
    fit: first fit the homogeneous (kappa0, mu0) to the data (qpat_fit_background),
    starting from the given pair; the pair used is returned in log["kappa0"], log["mu0"].
    step0_inner > 0: the zeroth step of Sec. 5 (PLSQR for kt alone, qpat_lsqr_init_kappa)
    with at most that many steps (and the window rule when m0, tau are given).
    discrepancy: None, or the factor of the noise level sqrt(n_ill N) below which
    an outer step's PLSQR run stops; log["discrepancy_fired"] records per outer
    step whether it did."""
    kind = {"pm": 0, "tvq": 1}[prior]
    N = ctx.N
    dev = chi.device
    beta = torch.zeros(2 * N, dtype=torch.float64, device=dev)
    beta_new = torch.zeros_like(beta)
    log = {"res_nl": [], "lsqr": [], "rejected": [], "pcg_iters": [], "discrepancy_fired": []}
    level = None if discrepancy is None else float(discrepancy) * math.sqrt(chi.numel())

    def setup_prior(b):
        if kind == 0:
            ctx.prior_setup(b[:N], b[N:], T, b_over_a, delta)
        else:
            ctx.prior_setup_r(b[:N], b[N:], kind, T, q, b_over_a, delta)

    def run_lsqr(count, noise_level=None):
        hist = [ctx.lsqr_residual()]
        iters = 0
        for m in range(1, count + 1):
            r, info = ctx.lsqr_step()
            hist.append(r)
            iters += info["iters_sum"]
            if noise_level is not None and r < noise_level:
                break
            if m0 is not None and tau is not None:
                rm = window_ratio(hist, m, m0)
                if rm is not None and rm <= tau:
                    break
        return hist, iters

    if fit:
        kappa0, mu0, log["fit_iters"], _ = ctx.fit_background(chi, W, kappa0, mu0)
    log["kappa0"], log["mu0"] = kappa0, mu0
    if beta0 is None:
        ctx.forward_log(kappa0, mu0, beta)          # homogeneous (kappa0, mu0)
        ctx.init_guess(chi, mu0, beta)
    else:
        beta.copy_(beta0)
    if step0_inner > 0:
        ctx.forward_log(kappa0, mu0, beta)
        setup_prior(beta)
        ctx.lsqr_init_kappa(chi, W, beta, beta_new)
        log["step0"], _ = run_lsqr(step0_inner)
        beta[:N] = beta_new[:N]
    ctx.forward_log(kappa0, mu0, beta)
    res = ctx.misfit(chi, W)
    for _ in range(outer):
        log["res_nl"].append(res)
        setup_prior(beta)
        ctx.lsqr_init(chi, W, beta, beta_new)
        hist, iters = run_lsqr(inner, level)
        log["lsqr"].append(hist)
        log["discrepancy_fired"].append(level is not None and hist[-1] < level)
        log["pcg_iters"].append(iters)
        ctx.forward_log(kappa0, mu0, beta_new)
        res_new = ctx.misfit(chi, W)
        rejected = res_new >= res
        log["rejected"].append(bool(rejected))
        if rejected and stop_on_reject:
            ctx.forward_log(kappa0, mu0, beta)      # restore the linearisation point
            log["res_nl"].append(res)
            return beta, log
        beta, beta_new = beta_new, beta
        res = res_new
    log["res_nl"].append(res)
    return beta, log


def finer_mesh_data(ctx_fine, kappa_fine, mu_fine, inj):
    """Noiseless data without the obvious inverse crime: h = mu phi from the
    forward solves of a context on the 2n mesh (qpat_forward), read at the
    reconstruction mesh's nodes (inj: their indices among the fine nodes, a
    device int64 tensor). Returns [n_ill][N_coarse] on the device."""
    h = torch.empty(ctx_fine.n_ill * ctx_fine.N, dtype=torch.float64, device=kappa_fine.device)
    ctx_fine.forward(kappa_fine, mu_fine, None, h)
    return h.view(ctx_fine.n_ill, ctx_fine.N).index_select(1, inj).contiguous()
