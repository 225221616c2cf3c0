"""Kuhn (Freudenthal) tetrahedral mesh of a voxel cube.

The cube [0, L]^3 is cut into n^3 voxels of side L/n. Node (i, j, k) has id
i + (n+1) * (j + (n+1) * k) (x fastest). Each voxel with lower corner v0 is
split into 6 tetrahedra, one per permutation s of the axes (x, y, z):
v0, v0 + e_s0, v0 + e_s0 + e_s1, v0 + (1, 1, 1). The split is conforming
between neighbouring voxels, every tetrahedron has volume (L/n)^3 / 6, and
each boundary square is cut along the diagonal that the tetrahedra use.

Boundary triangles are listed face by face in the order
-z, +z, -x, +x, -y, +y (tags 0..5).
"""
from dataclasses import dataclass
import numpy as np

FACE_NAMES = ("-z", "+z", "-x", "+x", "-y", "+y")

# axis permutations, fixed order
_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


@dataclass
class KuhnMesh:
    n: int
    L: float
    coords: np.ndarray      # [N][3] float64, mm
    tets: np.ndarray        # [E][4] int32
    bfaces: np.ndarray      # [F_b][3] int32
    bface_tag: np.ndarray   # [F_b] int8, cube face 0..5 in FACE_NAMES order

    @property
    def N(self):
        return self.coords.shape[0]

    @property
    def E(self):
        return self.tets.shape[0]

    @property
    def F_b(self):
        return self.bfaces.shape[0]

    @property
    def h(self):
        return self.L / self.n

    def node_index(self, i, j, k):
        m = self.n + 1
        return i + m * (j + m * k)


def kuhn_mesh(n: int, L: float = 40.0) -> KuhnMesh:
    if n < 1:
        raise ValueError("n must be >= 1")
    m = n + 1
    h = L / n
    g = np.arange(m, dtype=np.float64) * h
    # x fastest
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    coords = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)

    step = np.array([1, m, m * m], dtype=np.int64)
    vi = np.arange(n, dtype=np.int64)
    kk, jj, ii = np.meshgrid(vi, vi, vi, indexing="ij")
    v0 = (ii + m * (jj + m * kk)).ravel()  # voxel-major, x fastest
    far = step.sum()
    tets = np.empty((v0.size, 6, 4), dtype=np.int64)
    for p, (a, b, _) in enumerate(_PERMS):
        tets[:, p, 0] = v0
        tets[:, p, 1] = v0 + step[a]
        tets[:, p, 2] = v0 + step[a] + step[b]
        tets[:, p, 3] = v0 + far
    tets = tets.reshape(-1, 4).astype(np.int32)

    # boundary triangles, each boundary square split along its (+,+) diagonal
    sq = np.arange(n, dtype=np.int64)
    faces, tags = [], []

    def add_face(tag, fixed_axis, fixed_val, ax1, ax2):
        a2, a1 = np.meshgrid(sq, sq, indexing="ij")
        idx = np.zeros((3, a1.size), dtype=np.int64)
        idx[fixed_axis] = fixed_val
        idx[ax1] = a1.ravel()
        idx[ax2] = a2.ravel()
        base = idx[0] + m * (idx[1] + m * idx[2])
        d1, d2 = step[ax1], step[ax2]
        t1 = np.stack([base, base + d1, base + d1 + d2], axis=1)
        t2 = np.stack([base, base + d2, base + d1 + d2], axis=1)
        tri = np.stack([t1, t2], axis=1).reshape(-1, 3)
        faces.append(tri)
        tags.append(np.full(tri.shape[0], tag, dtype=np.int8))

    add_face(0, 2, 0, 0, 1)   # -z
    add_face(1, 2, n, 0, 1)   # +z
    add_face(2, 0, 0, 1, 2)   # -x
    add_face(3, 0, n, 1, 2)   # +x
    add_face(4, 1, 0, 0, 2)   # -y
    add_face(5, 1, n, 0, 2)   # +y
    bfaces = np.concatenate(faces).astype(np.int32)
    bface_tag = np.concatenate(tags)
    return KuhnMesh(n=n, L=float(L), coords=coords, tets=tets,
                    bfaces=bfaces, bface_tag=bface_tag)


def coarse_in_fine(n: int) -> np.ndarray:
    """Node indices, in the Kuhn mesh of 2n voxels per side, of the nodes of the
    mesh of n voxels per side on the same cube (node (i, j, k) of the coarse
    lattice is node (2i, 2j, 2k) of the fine one; both x fastest). The coarse
    Kuhn mesh's nodes are all fine nodes, so evaluating a fine P1 function at
    the coarse nodes is this index map."""
    m, mf = n + 1, 2 * n + 1
    i = 2 * np.arange(m, dtype=np.int64)
    kk, jj, ii = np.meshgrid(i, i, i, indexing="ij")
    return (ii + mf * (jj + mf * kk)).ravel()
