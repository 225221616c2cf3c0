"""Learned PCG initial guess: data from the solver, training, evaluation.

Every solve, network evaluation and training step is a libqpat call; the
host only generates the seeded phantoms (qpat_inputs) and sequences calls.

Samples: a seeded ellipsoid phantom with each of the context's
illuminations; the target is the fluence the solver returns. The network
input for illumination k is (log mu/mu0, log kappa/kappa0, log phi_hom_k),
phi_hom_k the fluence of the homogeneous (kappa0, mu0) medium.
"""
import time

import numpy as np
import torch

from qpat_inputs import ellipsoid_phantom, kappa_from_optics, rng


def _dev(a, device):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=torch.float64)


def homogeneous_fluence(ctx, kappa0, mu0, device):
    N = ctx.N
    phi = torch.empty(ctx.n_ill * N, dtype=torch.float64, device=device)
    ctx.forward(torch.full((N,), kappa0, dtype=torch.float64, device=device),
                torch.full((N,), mu0, dtype=torch.float64, device=device), phi)
    return phi


def make_samples(ctx, mesh, count, cfg_id, stream, device):
    """`count` seeded phantoms and their fluences for all illuminations."""
    g = rng(cfg_id, stream)
    out = []
    for _ in range(count):
        mua, mus, _ = ellipsoid_phantom(mesh.coords, g, L=mesh.L)
        kappa = _dev(kappa_from_optics(mua, mus), device)
        mu = _dev(mua, device)
        phi = torch.empty(ctx.n_ill * ctx.N, dtype=torch.float64, device=device)
        info = ctx.forward(kappa, mu, phi)
        out.append((kappa, mu, phi, info))
    return out


def train(ctx, samples, phi_hom, kappa0, mu0, epochs, lr, lr_decay=0.5, log=None):
    N, K = ctx.N, ctx.n_ill
    hist = []
    for ep in range(epochs):
        losses = []
        for kappa, mu, phi, _ in samples:
            for k in range(K):
                losses.append(ctx.guess_train(kappa, mu, kappa0, mu0, phi_hom[k * N:(k + 1) * N],
                                              phi[k * N:(k + 1) * N], lr))
        hist.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: mean loss {hist[-1]:.4e} (lr {lr:.2e})")
        lr *= lr_decay
    return hist


def evaluate(ctx, samples, phi_hom, kappa0, mu0, device):
    """PCG iterations and wall time per forward solve (all illuminations of a
    phantom in one block solve): zero start, homogeneous-fluence start, and
    the network's start. Same stopping rule in all three."""
    N, K = ctx.N, ctx.n_ill
    rows = []
    phi0 = torch.empty(K * N, dtype=torch.float64, device=device)
    out = torch.empty(K * N, dtype=torch.float64, device=device)
    for kappa, mu, _, _ in samples:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i0 = ctx.forward(kappa, mu, out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ih = ctx.forward_x0(kappa, mu, phi_hom, out)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ctx.guess_fluence(kappa, mu, kappa0, mu0, phi_hom, phi0)
        il = ctx.forward_x0(kappa, mu, phi0, out)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        rows.append(dict(zero_iters=i0["iters_sum"] / K, zero_ms=(t1 - t0) * 1e3,
                         hom_iters=ih["iters_sum"] / K, hom_ms=(t2 - t1) * 1e3,
                         net_iters=il["iters_sum"] / K, net_ms=(t3 - t2) * 1e3,
                         relres=max(i0["relres_max"], ih["relres_max"], il["relres_max"])))
    agg = {k: float(np.mean([r[k] for r in rows])) for k in rows[0]}
    agg["relres"] = float(max(r["relres"] for r in rows))
    return agg, rows
