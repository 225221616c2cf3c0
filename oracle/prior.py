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


class Prior:
    def __init__(self, geo, kt, mt, T=5e-3, b_over_a=1.0, delta=1e-6,
                 solver="direct", rtol=1e-10, kind="pm", q=1.0):
        self.Md = M_delta(geo, kt, mt, T, b_over_a, delta, kind, q)
        self._solve = make_solver(self.Md, solver, rtol)

    def apply(self, x):
        return self.Md @ x

    def solve(self, p):
        return self._solve(p)
