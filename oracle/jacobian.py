"""Forward map h(beta) and the Jacobian products J s, J^T t -- oracle.

Test infrastructure only (see the package docstring).

* Parametrisation (Sec. 3, eq. (3.1)): kappa = kappa0 exp(kt), mu = mu0 exp(mt)
  with beta = [kt; mt] in R^{2N}.
* Measurement (Sec. 2, eq. (2.2), nodal form in the Appendix):
  h_n = mu_n phi_n, one block of N per illumination, stacked (Sec. 4, the
  paragraph on several illuminations).
* J s and J^T t follow the Appendix literally: K phi = f, the load matrices
  G(1), G(2) are formed as sparse matrices, and

    J s   = diag(mu) K^{-1} (G(1) diag(kappa) s1 + G(2) diag(mu) s2)
            + diag(phi) diag(mu) s2,
    J^T t = [diag(kappa) G(1)^T K^{-1} diag(mu) t ;
             diag(mu) (G(2) K^{-1} diag(mu) t + diag(phi) t)],

  summed over illuminations for J^T.
"""
import numpy as np

from . import fem
from .solve import make_solver


def params(kappa0, mu0, beta):
    N = beta.size // 2
    return kappa0 * np.exp(beta[:N]), mu0 * np.exp(beta[N:])


class Linearisation:
    """Everything needed to apply h, J and J^T at one point (kappa, mu)."""

    def __init__(self, geo, kappa, mu, phi_src, solver="direct", rtol=1e-10):
        self.geo = geo
        self.kappa = np.asarray(kappa, dtype=np.float64)
        self.mu = np.asarray(mu, dtype=np.float64)
        self.K = fem.system_matrix(geo, self.kappa, self.mu)
        self.f = fem.load_vectors(geo, phi_src)
        self.solve = make_solver(self.K, solver, rtol)
        self.phi = np.atleast_2d(self.solve(self.f))        # [n_ill][N]
        self.h = self.mu[None, :] * self.phi
        self._G = {}

    @property
    def n_ill(self):
        return self.phi.shape[0]

    @property
    def N(self):
        return self.geo.N

    def G(self, k):
        if k not in self._G:
            self._G[k] = (fem.load_matrix_G1(self.geo, self.phi[k]),
                          fem.load_matrix_G2(self.geo, self.phi[k]))
        return self._G[k]

    def jvp(self, s):
        """J s for s = [s1; s2] in R^{2N}; returns [n_ill][N]."""
        N = self.N
        s1, s2 = s[:N], s[N:]
        out = np.empty((self.n_ill, N))
        for k in range(self.n_ill):
            G1, G2 = self.G(k)
            w = self.solve(G1 @ (self.kappa * s1) + G2 @ (self.mu * s2))
            out[k] = self.mu * w + self.phi[k] * self.mu * s2
        return out

    def vjp(self, t):
        """J^T t for t [n_ill][N]; returns R^{2N}."""
        t = np.atleast_2d(t)
        a1 = np.zeros(self.N)
        a2 = np.zeros(self.N)
        for k in range(self.n_ill):
            G1, G2 = self.G(k)
            z = self.solve(self.mu * t[k])
            a1 += G1.T @ z
            a2 += G2 @ z + self.phi[k] * t[k]
        return np.concatenate([self.kappa * a1, self.mu * a2])

    def dense_jacobian(self):
        """J column by column (tiny meshes only)."""
        n = 2 * self.N
        cols = [self.jvp(np.eye(1, n, j).ravel()).ravel() for j in range(n)]
        return np.stack(cols, axis=1)


def forward(geo, kappa, mu, phi_src, solver="direct", rtol=1e-10):
    lin = Linearisation(geo, kappa, mu, phi_src, solver, rtol)
    return lin.phi, lin.h
