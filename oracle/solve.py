"""Linear solves K x = b -- oracle.

Test infrastructure only (see the package docstring).

The paper applies K^{-1} (Appendix, "operate with the inverse of the FEM
system matrix") and M_delta^{-1} (Sec. 4, after eq. (4.10)) without naming a
method. Two independent routes are provided:

* ``direct``: a sparse LU factorisation (SuperLU) -- a library primitive;
* ``pcg``: textbook conjugate gradients preconditioned by the diagonal,
  started from x0 (default 0) and stopped when the TRUE residual satisfies
  ||b - K x||_2 <= rtol ||b||_2.
"""
import numpy as np
import scipy.sparse.linalg as spla


class Direct:
    """Factor once, solve many right-hand sides. symmetric=True orders the
    columns for the symmetric pattern (minimum degree on K + K^T) and pivots on
    the diagonal -- the same factorisation of an SPD matrix, with far less
    fill on 3D meshes than the default column ordering."""

    def __init__(self, K, symmetric=False):
        if symmetric:
            self.lu = spla.splu(K.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                                options=dict(SymmetricMode=True))
        else:
            self.lu = spla.splu(K.tocsc())

    def __call__(self, b):
        b = np.asarray(b, dtype=np.float64)
        if b.ndim == 1:
            return self.lu.solve(b)
        return np.stack([self.lu.solve(bi) for bi in b])


def pcg(K, b, rtol=1e-10, maxit=20000, x0=None, info=None):
    """Jacobi-preconditioned CG; returns x with ||b - K x|| <= rtol ||b|| (true residual)."""
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    if nb == 0.0:
        if info is not None:
            info.update(iters=0, relres=0.0)
        return np.zeros_like(b)
    dinv = 1.0 / K.diagonal()
    r = b - K @ x
    it = 0
    while True:
        z = dinv * r
        p = z.copy()
        rz = r @ z
        while np.linalg.norm(r) > rtol * nb and it < maxit:
            q = K @ p
            alpha = rz / (p @ q)
            x += alpha * p
            r -= alpha * q
            z = dinv * r
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
            it += 1
        r = b - K @ x                      # confirm on the true residual
        if np.linalg.norm(r) <= rtol * nb or it >= maxit:
            break
    relres = np.linalg.norm(r) / nb
    if info is not None:
        info.update(iters=it, relres=relres)
    if relres > rtol:
        raise RuntimeError(f"pcg: no convergence in {maxit} iterations (relres {relres:.3e})")
    return x


class Iterative:
    """K^{-1} by Jacobi-PCG at a fixed relative tolerance."""

    def __init__(self, K, rtol=1e-10, maxit=20000):
        self.K, self.rtol, self.maxit = K, rtol, maxit
        self.iters = []

    def __call__(self, b):
        b = np.asarray(b, dtype=np.float64)
        if b.ndim == 1:
            info = {}
            x = pcg(self.K, b, self.rtol, self.maxit, info=info)
            self.iters.append(info["iters"])
            return x
        return np.stack([self(bi) for bi in b])


def make_solver(K, method="direct", rtol=1e-10):
    if method == "direct":
        return Direct(K)
    if method == "direct_sym":
        return Direct(K, symmetric=True)
    if method == "pcg":
        return Iterative(K, rtol=rtol)
    raise ValueError(method)
