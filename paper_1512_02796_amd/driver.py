"""Algorithm 1 (Sec. 4) on the GPU library, with fixed or adaptive counts.

Host control flow only: every vector operation is a libqpat call (forward
solve, misfit, initial guess, prior assembly, LSQR). The host sees scalars
(residual norms) and decides what to call next.

  init  : kt = 0, mt = log(mean_k chi_k / phi0_k / mu0), phi0 the fluence of
          the homogeneous (kappa0, mu0) (preamble; several illuminations:
          paragraph after Algorithm 1 and Sec. 5)
  step 1: h = h(beta_l); yt = W (chi - h + J beta_l)     (inside qpat_lsqr_init)
  step 2: M_delta from kt_l, mt_l                          (qpat_prior_setup)
  step 3: PLSQR from 0: `inner` steps, or until r_m <= tau over a window of
          m0 steps (eq. (4.11)) when m0 and tau are given
  step 4: if ||W (chi - h(beta_{l+1}))|| >= ||W (chi - h(beta_l))|| the step
          is rejected; with stop_on_reject the previous iterate is returned,
          otherwise the comparison is only recorded.
"""
import torch


def window_ratio(history, m, m0):
    """r_m = 1 - res_m / res_{m-m0} for m > m0 (eq. (4.11)); history[0] = res_0."""
    if m <= m0:
        return None
    den = history[m - m0]
    return 1.0 - history[m] / den if den > 0 else 0.0


def reconstruct(ctx, chi, W, kappa0, mu0, outer, inner, T=5e-3, b_over_a=1.0, delta=1e-6,
                beta0=None, stop_on_reject=False, m0=None, tau=None, prior="pm", q=1.0):
    """prior: "pm" (Perona-Malik) or "tvq" (r(t) = T^(2-q) (t^2 + T^2)^(q/2) / q)."""
    kind = {"pm": 0, "tvq": 1}[prior]
    N = ctx.N
    dev = chi.device
    beta = torch.zeros(2 * N, dtype=torch.float64, device=dev)
    beta_new = torch.zeros_like(beta)
    if beta0 is None:
        ctx.forward_log(kappa0, mu0, beta)          # homogeneous (kappa0, mu0)
        ctx.init_guess(chi, mu0, beta)
    else:
        beta.copy_(beta0)
    log = {"res_nl": [], "lsqr": [], "rejected": [], "pcg_iters": []}
    ctx.forward_log(kappa0, mu0, beta)
    res = ctx.misfit(chi, W)
    for _ in range(outer):
        log["res_nl"].append(res)
        if kind == 0:
            ctx.prior_setup(beta[:N], beta[N:], T, b_over_a, delta)
        else:
            ctx.prior_setup_r(beta[:N], beta[N:], kind, T, q, b_over_a, delta)
        ctx.lsqr_init(chi, W, beta, beta_new)
        hist = [ctx.lsqr_residual()]
        iters = 0
        for m in range(1, inner + 1):
            r, info = ctx.lsqr_step()
            hist.append(r)
            iters += info["iters_sum"]
            if m0 is not None and tau is not None:
                rm = window_ratio(hist, m, m0)
                if rm is not None and rm <= tau:
                    break
        log["lsqr"].append(hist)
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
