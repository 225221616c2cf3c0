"""Priorconditioned LSQR -- oracle.

Test infrastructure only (see the package docstring).

Sec. 4 solves (L^{-1})^T A^T A L^{-1} bt = (L^{-1})^T A^T yt (eq. (4.10)),
beta = L^{-1} bt, with LSQR started from bt = 0, where M_delta = L^T L is only
formal: only products with M_delta^{-1} are available.

This is Paige and Saunders' LSQR (their bidiagonalisation and the Givens
update of the solution) applied to Abar = A L^{-1}, written in the variables
v = L^{-1} vbar, w = L^{-1} wbar, x = L^{-1} xbar and what = M_delta v, so that
L never appears:

  beta_1 u = yt
  p = A^T u;            r = M_delta^{-1} p;  alpha = sqrt(p.r)
  v = r / alpha;        what = p / alpha;    w = v
  phibar = beta_1;      rhobar = alpha
  each step:
    q = A v - alpha u;        beta = ||q||;   u = q / beta
    p = A^T u - beta what;    r = M_delta^{-1} p;  alpha = sqrt(p.r)
    v = r / alpha;            what = p / alpha
    rho = hypot(rhobar, beta); c = rhobar/rho; s = beta/rho
    theta = s alpha; rhobar = -c alpha; phi = c phibar; phibar = s phibar
    x += (phi/rho) w;         w = v - (theta/rho) w
  |phibar| = ||A x - yt|| (exact arithmetic), and x is already beta.

The iterate therefore stays in range(M_delta^{-1}) as Sec. 4 notes.

Option ``reorth`` (default on): before normalising, q is orthogonalised
against all earlier u_j, and p against all earlier vbar_j = L v_j in the
form p -= (v_j . p) what_j (since vbar_j . L^{-T} p = v_j . p and
L^T vbar_j = what_j), each by classical Gram-Schmidt applied twice. In exact
arithmetic this changes nothing; in floating point it keeps both bases
orthonormal, which plain LSQR loses on this strongly graded operator.
"""
import numpy as np


class PLSQR:
    def __init__(self, A, At, Minv, yt, reorth=True):
        self.A, self.At, self.Minv = A, At, Minv
        self.reorth = reorth
        yt = np.asarray(yt, dtype=np.float64)
        self.beta1 = np.linalg.norm(yt)
        self.steps = 0
        self.done = self.beta1 == 0.0
        self.U, self.V, self.WH = [], [], []
        if self.done:
            self.x = np.zeros(self.At(np.zeros_like(yt)).size)
            self.phibar = 0.0
            self.history = [0.0]
            return
        self.u = yt / self.beta1
        p = self.At(self.u)
        r = self.Minv(p)
        self.alpha = np.sqrt(p @ r)
        self.x = np.zeros_like(p)
        if self.alpha == 0.0:
            self.done = True
            self.v = self.w = self.what = np.zeros_like(p)
        else:
            self.v = r / self.alpha
            self.what = p / self.alpha
            self.w = self.v.copy()
        if reorth:
            self.U.append(self.u)
            self.V.append(self.v)
            self.WH.append(self.what)
        self.phibar = self.beta1
        self.rhobar = self.alpha
        self.history = [self.phibar]

    def _orth_u(self, q):
        for _ in range(2):
            c = [uj @ q for uj in self.U]
            for cj, uj in zip(c, self.U):
                q = q - cj * uj
        return q

    def _orth_p(self, p):
        for _ in range(2):
            c = [vj @ p for vj in self.V]
            for cj, wj in zip(c, self.WH):
                p = p - cj * wj
        return p

    def step(self):
        """One LSQR step; returns the residual estimate |phibar|."""
        if self.done:
            self.history.append(abs(self.phibar))
            return abs(self.phibar)
        q = self.A(self.v) - self.alpha * self.u
        if self.reorth:
            q = self._orth_u(q)
        beta = np.linalg.norm(q)
        if beta == 0.0:
            # Abar xbar = yt is solved within the current Krylov space
            self.x = self.x + (self.phibar / self.rhobar) * self.w
            self.phibar = 0.0
            self.done = True
            self.steps += 1
            self.history.append(0.0)
            return 0.0
        self.u = q / beta
        p = self.At(self.u) - beta * self.what
        if self.reorth:
            p = self._orth_p(p)
        r = self.Minv(p)
        pr = p @ r
        if pr < 0.0 or not np.isfinite(pr):
            raise FloatingPointError("PLSQR breakdown: p.r <= 0")
        alpha = np.sqrt(pr)
        rho = np.hypot(self.rhobar, beta)
        c = self.rhobar / rho
        s = beta / rho
        theta = s * alpha
        self.rhobar = -c * alpha
        phi = c * self.phibar
        self.phibar = s * self.phibar
        self.x = self.x + (phi / rho) * self.w
        if alpha == 0.0:
            self.done = True
            self.w = np.zeros_like(self.w)
        else:
            v = r / alpha
            self.what = p / alpha
            self.w = v - (theta / rho) * self.w
            self.v = v
            if self.reorth:
                self.U.append(self.u)
                self.V.append(self.v)
                self.WH.append(self.what)
        self.alpha = alpha
        self.steps += 1
        self.history.append(abs(self.phibar))
        return abs(self.phibar)


def window_ratio(history, m, m0):
    """r_m = 1 - res_m / res_{m-m0}, defined for m > m0 (Sec. 4, eq. (4.11))."""
    if m <= m0:
        return None
    den = history[m - m0]
    return 1.0 - history[m] / den if den > 0 else 0.0


def discrepancy_reached(history, m, level):
    """Morozov's discrepancy principle (Sec. 4, the remark after Algorithm 1):
    the residual of the linearised model after m steps has fallen below the
    whitened noise level, res_m < level (level = sqrt(K N) for K illuminations
    of N nodes, times an optional factor)."""
    return history[m] < level


def plsqr(A, At, Minv, yt, iters, m0=None, tau=None, reorth=True, noise_level=None):
    """Run a fixed number of steps, or stop early once r_m <= tau when m0, tau
    given, or once the residual is below noise_level when that is given (the
    discrepancy principle); the first rule that fires ends the run."""
    it = PLSQR(A, At, Minv, yt, reorth=reorth)
    for m in range(1, iters + 1):
        it.step()
        if noise_level is not None and discrepancy_reached(it.history, m, noise_level):
            break
        if m0 is not None and tau is not None:
            rm = window_ratio(it.history, m, m0)
            if rm is not None and rm <= tau:
                break
    return it
