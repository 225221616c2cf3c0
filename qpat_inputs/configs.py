"""Workload recipes.

C1..C5 are the five reconstruction workloads (ids 1..5): a 40 mm cube cut
into n^3 Kuhn voxels, seeded phantoms, face or Gaussian sources. Small
variants (ids >= 100) reuse the same generators at sizes the FP64 oracle
finishes in seconds.

Method constants (Section 4, the choices stated after Algorithm 1):
T = 5e-3, delta = 1e-6, b/a = 1, m0 = 10, tau = 1e-2.
"""
from dataclasses import dataclass, field
import numpy as np

from .mesh import kuhn_mesh, KuhnMesh
from .phantom import (sphere_phantom, ellipsoid_phantom, kappa_from_optics,
                      BG_MUA, BG_MUS)
from .sources import face_sources, gaussian_sources


def rng(cfg_id, stream):
    return np.random.default_rng([1512, int(cfg_id), int(stream)])


CONFIGS = {
    # plain FP64: 16^3 voxels, 4 unit face sources (-z,+z,-x,+x), two spheres
    "C1": dict(id=1, n=16, n_ill=4, source="face", phantom="spheres",
               noise=0.01, outer=5, inner=20, precision="fp64"),
    # plain FP64 on one GPU: 64^3, 8 Gaussian sources, 6 ellipsoids
    "C2": dict(id=2, n=64, n_ill=8, source="gauss", phantom="ellipsoids",
               noise=0.02, outer=3, inner=30, precision="fp64"),
    # batched + mixed: 128^3, 16 Gaussian sources in one block solve
    "C3": dict(id=3, n=128, n_ill=16, source="gauss", phantom="ellipsoids",
               noise=0.02, outer=3, inner=30, precision="mixed"),
    # batched instances: template of the 32 uneven instances (sizes from batch_instances)
    "C4": dict(id=4, n=48, n_ill=8, source="gauss", phantom="ellipsoids",
               noise=0.02, outer=3, inner=30, precision="mixed"),
    # learned initial guess: 96^3, 8 illuminations
    "C5": dict(id=5, n=96, n_ill=8, source="gauss", phantom="ellipsoids",
               noise=0.02, outer=3, inner=30, precision="mixed"),
    # small variants for parity tests
    "T4": dict(id=104, n=4, n_ill=2, source="face", phantom="spheres",
               noise=0.01, outer=2, inner=5, precision="fp64"),
    "T8": dict(id=108, n=8, n_ill=4, source="gauss", phantom="ellipsoids",
               noise=0.01, outer=2, inner=10, precision="fp64"),
    "T12": dict(id=112, n=12, n_ill=3, source="gauss", phantom="ellipsoids",
                noise=0.01, outer=2, inner=10, precision="fp64"),
    "T24": dict(id=124, n=24, n_ill=6, source="gauss", phantom="ellipsoids",
                noise=0.02, outer=2, inner=10, precision="fp64"),
    # illumination study on a small cube (Sec. 5, second test: 1, 2 or 3 face
    # illuminations; its inclusion sizes are not given, so two seeded ellipsoids
    # sized for an 11 mm cube), data simulated on the 2n mesh and injected
    "S2": dict(id=7, n=32, n_ill=3, source="face", phantom="ellipsoids", L=11.0, count=2,
               axes=(1.0, 2.5), noise=0.01, outer=3, inner=30, precision="fp64"),
}

METHOD = dict(T=5e-3, delta=1e-6, b_over_a=1.0, m0=10, tau=1e-2, pcg_rtol=1e-10)


def batch_instances(count=32, cfg_id=4):
    """Sizes of the batched-instance workload: n ~ U{24..96} voxels per side,
    n_ill ~ U{4..12}, drawn from stream 6; instance i uses phantom id 1000 cfg_id + i."""
    g = rng(cfg_id, 6)
    n = g.integers(24, 97, size=count)
    k = g.integers(4, 13, size=count)
    return [dict(n=int(n[i]), n_ill=int(k[i]), id=1000 * int(cfg_id) + i) for i in range(count)]


def config(name, **over):
    c = dict(CONFIGS[name])
    c.update(over)
    c["name"] = name
    return c


@dataclass
class Problem:
    cfg: dict
    mesh: KuhnMesh
    mua: np.ndarray
    mus: np.ndarray
    kappa: np.ndarray          # true nodal diffusion
    mu: np.ndarray             # true nodal absorption (= mua)
    phi_src: np.ndarray        # [n_ill][F_b][3]
    kappa0: float = 1.0 / (3.0 * (BG_MUA + BG_MUS))
    mu0: float = BG_MUA
    method: dict = field(default_factory=lambda: dict(METHOD))
    shapes: object = None

    @property
    def n_ill(self):
        return self.phi_src.shape[0]


def make_problem(name, L=40.0, **over):
    c = config(name, **over)
    L = c.get("L", L)
    mesh = kuhn_mesh(c["n"], L)
    g = rng(c["id"], 0)
    if c["phantom"] == "spheres":
        mua, mus, shapes = sphere_phantom(mesh.coords, g, L=L)
    elif c["phantom"] == "ellipsoids":
        kw = {k: c[k] for k in ("count", "axes") if k in c}
        mua, mus, shapes = ellipsoid_phantom(mesh.coords, g, L=L, **kw)
    elif c["phantom"] == "background":
        mua = np.full(mesh.N, BG_MUA)
        mus = np.full(mesh.N, BG_MUS)
        shapes = None
    else:
        raise ValueError(c["phantom"])
    if c["source"] == "face":
        faces = list(range(c["n_ill"]))     # -z, +z, -x, +x, -y, +y
        phi_src = face_sources(mesh, faces)
    else:
        phi_src = gaussian_sources(mesh, c["n_ill"])
    kappa = kappa_from_optics(mua, mus)
    return Problem(cfg=c, mesh=mesh, mua=mua, mus=mus, kappa=kappa, mu=mua.copy(),
                   phi_src=phi_src, shapes=shapes)
