"""Boundary photon-flux sources as values at boundary-triangle vertices.

A source is stored per triangle vertex, shape [n_ill][F_b][3], so a flux
that jumps across a cube edge (an indicator of one face) is represented
exactly by a piecewise-linear function on each boundary triangle.
"""
import numpy as np

from .mesh import FACE_NAMES

# unit tangent axes (in-plane coordinates) of each cube face, -z,+z,-x,+x,-y,+y
_FACE_AXIS = (2, 2, 0, 0, 1, 1)
_FACE_SIDE = (0, 1, 0, 1, 0, 1)
_FACE_TANGENTS = {2: (0, 1), 0: (1, 2), 1: (0, 2)}


def face_sources(mesh, faces):
    """Unit indicator source on each listed cube face (tags in FACE_NAMES order)."""
    out = np.zeros((len(faces), mesh.F_b, 3))
    for k, f in enumerate(faces):
        out[k, mesh.bface_tag == f, :] = 1.0
    return out


def gaussian_centre(mesh, k):
    """Centre of Gaussian source k: face k mod 6; ring k // 6 shifts the
    centre by (0,0), (+L/4, 0), (0, +L/4) in the face's tangent axes."""
    L = mesh.L
    face = k % 6
    ring = (k // 6) % 3
    axis = _FACE_AXIS[face]
    c = np.full(3, L / 2.0)
    c[axis] = L * _FACE_SIDE[face]
    t1, t2 = _FACE_TANGENTS[axis]
    if ring == 1:
        c[t1] += L / 4.0
    elif ring == 2:
        c[t2] += L / 4.0
    return face, c


def gaussian_sources(mesh, n_ill, sigma=5.0, amplitude=1.0):
    """n_ill Gaussian spots exp(-|x-c|^2 / (2 sigma^2)) on cube faces, sampled at
    the vertices of that face's triangles; zero on the other faces."""
    out = np.zeros((n_ill, mesh.F_b, 3))
    for k in range(n_ill):
        face, c = gaussian_centre(mesh, k)
        sel = mesh.bface_tag == face
        pts = mesh.coords[mesh.bfaces[sel]]          # [f][3][3]
        d2 = np.sum((pts - c) ** 2, axis=2)
        out[k, sel, :] = amplitude * np.exp(-d2 / (2.0 * sigma * sigma))
    return out


__all__ = ["face_sources", "gaussian_sources", "gaussian_centre", "FACE_NAMES"]
