"""Seeded optical phantoms sampled at mesh nodes.

A node lies inside a sphere when its distance to the centre is at most the
radius, and inside an ellipsoid when its body-frame coordinates satisfy
sum (x_i / a_i)^2 <= 1. Later shapes overwrite earlier ones. The diffusion
coefficient follows from absorption and reduced scattering as
kappa = 1 / (3 (mu_a + mu_s')), the usual diffusion-approximation relation.
"""
import numpy as np

BG_MUA = 0.01     # mm^-1
BG_MUS = 1.0      # mm^-1 (reduced scattering)


def kappa_from_optics(mua, mus):
    return 1.0 / (3.0 * (mua + mus))


def background_phantom(coords, mua=BG_MUA, mus=BG_MUS):
    N = coords.shape[0]
    return np.full(N, float(mua)), np.full(N, float(mus))


def sphere_phantom(coords, rng, L=40.0, count=2, radius=5.0, lo=8.0, hi=32.0,
                   min_sep=12.0, mua_in=0.02, mus_in=2.0):
    """Spheres with centres U[lo, hi]^3, redrawn until pairwise >= min_sep apart."""
    mua, mus = background_phantom(coords)
    centres = []
    while len(centres) < count:
        c = rng.uniform(lo, hi, size=3)
        if all(np.linalg.norm(c - d) >= min_sep for d in centres):
            centres.append(c)
    for c in centres:
        inside = np.sum((coords - c) ** 2, axis=1) <= radius * radius
        mua[inside] = mua_in
        mus[inside] = mus_in
    return mua, mus, np.array(centres)


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def ellipsoid_phantom(coords, rng, L=40.0, count=6, axes=(2.5, 8.0),
                      mua_range=(0.005, 0.03), mus_range=(0.5, 2.0)):
    """Ellipsoids with semi-axes U[axes], uniform random orientation, centres
    at least the largest semi-axis away from the boundary."""
    mua, mus = background_phantom(coords)
    shapes = []
    for _ in range(count):
        a = rng.uniform(axes[0], axes[1], size=3)
        R = _random_rotation(rng)
        margin = a.max()
        c = rng.uniform(margin, L - margin, size=3)
        va = rng.uniform(*mua_range)
        vs = rng.uniform(*mus_range)
        body = (coords - c) @ R          # body-frame coordinates
        inside = np.sum((body / a) ** 2, axis=1) <= 1.0
        mua[inside] = va
        mus[inside] = vs
        shapes.append(dict(centre=c, axes=a, rot=R, mua=va, mus=vs))
    return mua, mus, shapes
