"""Seeded Gaussian draws: noise draws and test vectors for J and J^T."""
import numpy as np

from .configs import rng


def noise_draws(cfg_id, n_ill, N):
    """Standard normal draws xi [n_ill][N] (stream 1); noise is sigma_rel*|h|*xi."""
    return rng(cfg_id, 1).standard_normal((n_ill, N))


def probe_vectors(cfg_id, n_ill, N):
    """s ~ N(0,1) of length 2N and t ~ N(0,1) of shape [n_ill][N] (stream 2)."""
    g = rng(cfg_id, 2)
    s = g.standard_normal(2 * N)
    t = g.standard_normal((n_ill, N))
    return s, t
