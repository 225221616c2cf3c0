"""Seeded synthetic inputs shared by the FP64 oracle and the GPU library.

This module builds meshes, phantoms, boundary sources, Gaussian draws and
test vectors. It holds none of the reconstruction method's arithmetic
(no assembly, no solve, no Jacobian, no prior): everything here is input
that a user of the method would also have to supply.

Random streams: ``numpy.random.default_rng([1512, cfg, stream])`` with
stream 0 = phantom, 1 = noise draws, 2 = test vectors s and t,
3 = training samples of the learned guess, 4 = held-out samples, 5 = initial
network weights, 6 = sizes of the batched instances.
"""
from .mesh import kuhn_mesh, KuhnMesh, FACE_NAMES, coarse_in_fine
from .phantom import (sphere_phantom, ellipsoid_phantom, background_phantom,
                      kappa_from_optics)
from .sources import face_sources, gaussian_sources
from .configs import CONFIGS, config, rng, make_problem, Problem, batch_instances
from .vectors import probe_vectors, noise_draws
from .net import initial_params

__all__ = [
    "kuhn_mesh", "KuhnMesh", "FACE_NAMES", "sphere_phantom", "ellipsoid_phantom",
    "background_phantom", "kappa_from_optics", "face_sources", "gaussian_sources",
    "CONFIGS", "config", "rng", "make_problem", "Problem", "batch_instances", "probe_vectors", "noise_draws", "initial_params",
]
