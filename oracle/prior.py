"""Lagged-diffusivity TV-type prior matrix M_delta -- oracle.

Test infrastructure only (see the package docstring).

* R(u) = int r(|grad u|) dx (Sec. 3, eq. (3.6)) with either
  - Perona-Malik, r(t) = (T^2/2) log(1 + (t/T)^2) (eq. (3.7)), kind "pm", or
  - TV^q, r(t) = T^(2-q) (t^2 + T^2)^(q/2) / q, kind "tvq" (the remark after
    eq. (3.7): smoothed TV, q = 1, and TV^q fit the same algorithm). The
    factor T^(2-q) makes c(0) = 1 as for Perona-Malik; a constant factor of
    r only rescales the free weights a, b.
* grad R(u) = M(u) u, where M(u) is the FEM matrix of -div(c_u grad .) with a
  natural boundary condition and c_u = r'(|grad u|) / |grad u|
  (Sec. 4, eq. (4.3) and the text around it). For P1 u the gradient is
  constant on each tetrahedron, so c_u is too.
* Lagged diffusivity freezes c at the current iterate; the block matrix
  M = blockdiag(M(kt), (b/a) M(mt)) (eq. (4.5)) is shifted to
  M_delta = M + delta I (eq. (4.8)).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import _assemble
from .solve import make_solver


def r_of(t, T, kind="pm", q=1.0):
    """r(t) itself (the prior's integrand)."""
    t = np.asarray(t, dtype=np.float64)
    if kind == "pm":
        return 0.5 * T * T * np.log1p((t / T) ** 2)
    if kind == "tvq":
        return T ** (2.0 - q) * (t * t + T * T) ** (q / 2.0) / q
    raise ValueError(kind)


def r_prime(t, T, kind="pm", q=1.0):
    """r'(t) for the chosen r."""
    t = np.asarray(t, dtype=np.float64)
    if kind == "pm":
        return t / (1.0 + (t / T) ** 2)
    if kind == "tvq":
        return T ** (2.0 - q) * t * (t * t + T * T) ** (q / 2.0 - 1.0)
    raise ValueError(kind)


def diffusivity(t, T, kind="pm", q=1.0):
    """c = r'(t)/t, with its limit 1 at t = 0 (both kinds)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.ones_like(t)
    nz = t > 0
    out[nz] = r_prime(t[nz], T, kind, q) / t[nz]
    return out


def R_of(geo, u, T, kind="pm", q=1.0):
    """R(u) = sum over tetrahedra of |T| r(|grad u_T|) for a nodal P1 field u."""
    return float(np.sum(geo.vol * r_of(np.linalg.norm(tet_gradients(geo, u), axis=1), T, kind, q)))


def tet_gradients(geo, u):
    """grad u on each tetrahedron for a nodal P1 field u: [E][3]."""
    return np.einsum("ea,eai->ei", u[geo.tets], geo.grad)


def M_of(geo, u, T, kind="pm", q=1.0):
    """M(u)_ij = int c_u grad(phi_i).grad(phi_j) dx."""
    c = diffusivity(np.linalg.norm(tet_gradients(geo, u), axis=1), T, kind, q)
    gg = np.einsum("eai,ebi->eab", geo.grad, geo.grad)
    return _assemble(geo.N, geo.tets, (c * geo.vol)[:, None, None] * gg)


def M_delta(geo, kt, mt, T=5e-3, b_over_a=1.0, delta=1e-6, kind="pm", q=1.0):
    """M_delta = blockdiag(M(kt), (b/a) M(mt)) + delta I  (2N x 2N)."""
    Mk = M_of(geo, kt, T, kind, q)
    Mm = M_of(geo, mt, T, kind, q)
    return (sp.block_diag([Mk, b_over_a * Mm]) + delta * sp.identity(2 * geo.N)).tocsr()


class DeflatedDirect:
    """r = M_delta^{-1} p with the delta-eigenvector of each block taken exactly.

    Each diagonal block D = c M(u) + delta I of M_delta (eq. (4.8); c = 1 for
    kt, b/a for mt, eq. (4.5)) has c M(u) 1 = 0: M(u) is the stiffness matrix
    of -div(c_u grad) with a natural boundary condition, whose rows sum to
    zero. Hence D 1 = delta 1, and as D is symmetric it maps the mean-free
    vectors onto themselves. With m = mean(p):

        r = (m / delta) 1 + y,   D y = p - m 1,   mean(y) = 0.

    y comes from a sparse LU factorisation of D; the LU's rounding error along
    1 is amplified by 1/delta, so y's mean -- zero in exact arithmetic -- is
    removed. What remains is the error of D on the mean-free vectors, whose
    smallest eigenvalue is far above delta."""

    def __init__(self, Md, N, delta):
        Md = Md.tocsr()
        self.N, self.delta = N, float(delta)
        self.nb = Md.shape[0] // N          # diagonal blocks of N (2 for M_delta, 1 for one block)
        self.lus = [spla.splu(Md[j * N:(j + 1) * N, j * N:(j + 1) * N].tocsc()) for j in range(self.nb)]

    def __call__(self, p):
        p = np.asarray(p, dtype=np.float64)
        N = self.N
        out = np.empty(self.nb * N)
        for j in range(self.nb):
            pj = p[j * N:(j + 1) * N]
            m = pj.mean()
            y = self.lus[j].solve(pj - m)
            out[j * N:(j + 1) * N] = (y - y.mean()) + m / self.delta
        return out


class Prior:
    """M_delta at (kt, mt) and its inverse. solver: "direct" (sparse LU of
    the whole matrix), "pcg" (Jacobi-PCG) or "deflated" (DeflatedDirect)."""

    def __init__(self, geo, kt, mt, T=5e-3, b_over_a=1.0, delta=1e-6,
                 solver="direct", rtol=1e-10, kind="pm", q=1.0):
        self.Md = M_delta(geo, kt, mt, T, b_over_a, delta, kind, q)
        if solver == "deflated":
            self._solve = DeflatedDirect(self.Md, geo.N, delta)
        else:
            self._solve = make_solver(self.Md, solver, rtol)

    def apply(self, x):
        return self.Md @ x

    def solve(self, p):
        return self._solve(p)
