"""P1 finite elements of the diffusion approximation -- oracle.

Test infrastructure only (see the package docstring).

Model (Sec. 2, eq. (2.1)): -div(kappa grad phi) + mu phi = 0 in Omega,
phi/4 + (1/2) kappa d(phi)/d(nu) = Phi on the boundary. Its weak form
(Appendix) is

    int kappa grad(phi).grad(v) + mu phi v dx + 1/2 int_bdry phi v dS
        = 2 int_bdry Phi v dS,

which gives the system matrix K(kappa, mu) and the load vector f(Phi).
kappa and mu enter as the P1 interpolants of their nodal values (the
parametrisation of Sec. 3, eqs. (3.1)-(3.2), puts the log-parameters in the
P1 basis; the nodal kappa, mu are their pointwise images).

Every integral is evaluated by a quadrature rule that is exact for the
integrand's polynomial degree: a 5-point degree-3 rule on tetrahedra and the
3-point edge-midpoint degree-2 rule on triangles. No closed-form element
matrix is used here.
"""
from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp

# degree-3 tetrahedral rule in barycentric coordinates, weights relative to |T|
# (centroid weight -4/5, four points (1/2, 1/6, 1/6, 1/6) with weight 9/20).
_TET_PTS = np.array([[0.25, 0.25, 0.25, 0.25],
                     [0.5, 1 / 6, 1 / 6, 1 / 6],
                     [1 / 6, 0.5, 1 / 6, 1 / 6],
                     [1 / 6, 1 / 6, 0.5, 1 / 6],
                     [1 / 6, 1 / 6, 1 / 6, 0.5]])
_TET_W = np.array([-0.8, 0.45, 0.45, 0.45, 0.45])

# degree-2 triangle rule: edge midpoints, weights 1/3 relative to |F|
_TRI_PTS = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])
_TRI_W = np.array([1 / 3, 1 / 3, 1 / 3])


@dataclass
class Geometry:
    N: int
    tets: np.ndarray     # [E][4]
    vol: np.ndarray      # [E]   |T|
    grad: np.ndarray     # [E][4][3]  gradients of the barycentric coordinates
    bfaces: np.ndarray   # [F][3]
    area: np.ndarray     # [F]   |F|


def geometry(coords, tets, bfaces):
    """|T| and grad(lambda_a) of every tetrahedron, |F| of every boundary triangle."""
    tets = np.asarray(tets, dtype=np.int64)
    bfaces = np.asarray(bfaces, dtype=np.int64)
    x = coords[tets]                           # [E][4][3]
    D = x[:, 1:, :] - x[:, :1, :]              # rows: edges from vertex 0
    det = np.linalg.det(D)
    if np.any(np.abs(det) <= 1e-14 * np.max(np.abs(D)) ** 3):
        raise ValueError("degenerate tetrahedron")
    Dinv = np.linalg.inv(D)                    # lambda_{1..3} = Dinv^T (x - x0)
    g = np.empty((tets.shape[0], 4, 3))
    g[:, 1:, :] = np.transpose(Dinv, (0, 2, 1))
    g[:, 0, :] = -g[:, 1:, :].sum(axis=1)
    vol = np.abs(det) / 6.0
    y = coords[bfaces]
    area = 0.5 * np.linalg.norm(np.cross(y[:, 1] - y[:, 0], y[:, 2] - y[:, 0]), axis=1)
    return Geometry(N=coords.shape[0], tets=tets, vol=vol, grad=g, bfaces=bfaces, area=area)


def _assemble(N, conn, elem):
    """Sum element matrices elem [E][k][k] over connectivity conn [E][k]."""
    k = conn.shape[1]
    rows = np.repeat(conn, k, axis=1).ravel()
    cols = np.tile(conn, (1, k)).ravel()
    return sp.coo_matrix((elem.reshape(-1), (rows, cols)), shape=(N, N)).tocsr()


def _tet_interp(geo, nodal):
    """P1 interpolant of a nodal field at the tetrahedral quadrature points: [E][Q]."""
    return nodal[geo.tets] @ _TET_PTS.T


def stiffness(geo, coef):
    """S(coef)_ij = int coef_h grad(phi_i).grad(phi_j) dx."""
    cq = _tet_interp(geo, coef)                        # [E][Q]
    integral = geo.vol * (cq @ _TET_W)                 # int_T coef_h
    gg = np.einsum("eai,ebi->eab", geo.grad, geo.grad)
    return _assemble(geo.N, geo.tets, integral[:, None, None] * gg)


def mass(geo, coef):
    """Mass(coef)_ij = int coef_h phi_i phi_j dx."""
    cq = _tet_interp(geo, coef)                        # [E][Q]
    lam = _TET_PTS                                     # [Q][4]
    elem = np.einsum("q,eq,qa,qb->eab", _TET_W, cq, lam, lam) * geo.vol[:, None, None]
    return _assemble(geo.N, geo.tets, elem)


def boundary_mass(geo):
    """B_ij = int_bdry phi_i phi_j dS."""
    lam = _TRI_PTS
    elem = np.einsum("q,qa,qb->ab", _TRI_W, lam, lam)[None] * geo.area[:, None, None]
    return _assemble(geo.N, geo.bfaces, elem)


def system_matrix(geo, kappa, mu):
    """K(kappa, mu) = S(kappa) + Mass(mu) + (1/2) B (Appendix, weak form)."""
    return (stiffness(geo, kappa) + mass(geo, mu) + 0.5 * boundary_mass(geo)).tocsr()


def load_vectors(geo, phi_src):
    """f_i = 2 int_bdry Phi_h phi_i dS for each illumination; phi_src [n_ill][F][3]
    holds Phi at the vertices of each boundary triangle."""
    phi_src = np.atleast_3d(phi_src)
    n_ill = phi_src.shape[0]
    lam = _TRI_PTS                                     # [Q][3]
    f = np.zeros((n_ill, geo.N))
    for k in range(n_ill):
        Phi_q = phi_src[k] @ lam.T                     # [F][Q]
        elem = 2.0 * np.einsum("q,fq,qa->fa", _TRI_W, Phi_q, lam) * geo.area[:, None]
        np.add.at(f[k], geo.bfaces.ravel(), elem.ravel())
    return f


def load_matrix_G1(geo, phi):
    """G(1)_ij = - int phi_j grad(phi_h).grad(phi_i) dx (Appendix)."""
    grad_phi = np.einsum("ea,eai->ei", phi[geo.tets], geo.grad)          # [E][3]
    gi = np.einsum("ei,eai->ea", grad_phi, geo.grad)                      # grad phi . grad phi_i
    int_lam = geo.vol[:, None] * (_TET_W @ _TET_PTS)[None, :]             # int_T phi_j
    elem = -gi[:, :, None] * int_lam[:, None, :]                          # [E][i][j]
    return _assemble(geo.N, geo.tets, elem)


def load_matrix_G2(geo, phi):
    """G(2)_ij = - int phi_j phi_h phi_i dx (Appendix)."""
    return -mass(geo, phi)
