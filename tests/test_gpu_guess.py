"""Learned initial guess: the MFMA conv net against the FP64 oracle, training,
and forward solves started from a guess.

Inputs and weights are drawn from a seeded generator and rounded to BF16 on
the host, so both sides see the same numbers. The library keeps hidden
activations and backward signals in BF16 (unit roundoff 2^-8 = 3.9e-3) with
FP32 accumulation; through three hidden layers that gives relative errors of
about 1e-2 in the output and the gradients, hence the 3e-2 bounds.
"""
import numpy as np
import pytest
import torch

from gpu_util import GpuProblem, dev, host, rel, need_gpu, assert_close
from oracle import convnet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def bf16_round(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def flat_params(params):
    out = []
    for w, b in params:
        out.append(w.ravel())
        out.append(b.ravel())
    return np.concatenate(out)


def lattice_ctx(nx, ny, nz):
    """A context on the Kuhn mesh whose node lattice is nx x ny x nz."""
    from paper_1512_02796_amd import qpat
    from qpat_inputs import kuhn_mesh
    assert nx == ny == nz
    m = kuhn_mesh(nx - 1, 40.0)
    ctx = qpat.Context(dev(m.coords), dev(m.tets, torch.int32), dev(m.bfaces, torch.int32))
    ctx.guess_setup(nx, ny, nz)
    return ctx, m


def seeded_net(seed, shape):
    rng = np.random.default_rng(seed)
    params = convnet.init_params(rng)
    for i, (w, b) in enumerate(params):
        params[i] = [bf16_round(w), (0.05 * rng.standard_normal(b.shape)).astype(np.float32).astype(np.float64)]
    x = bf16_round(rng.standard_normal((3,) + shape))
    return params, x


@pytest.mark.parametrize("n", [9, 12])
def test_net_forward_matches_oracle(n):
    ctx, m = lattice_ctx(n, n, n)
    params, x = seeded_net(n, (n, n, n))
    ctx.guess_set_params(dev(flat_params(params), torch.float32))
    out = torch.empty(m.N, dtype=torch.float32, device="cuda")
    ctx.guess_eval(dev(x.reshape(3, -1), torch.float32), out)
    ref, _ = convnet.forward(params, x)
    assert_close(host(out).astype(np.float64), ref.ravel(), 3e-2, f"net output n={n}")
    # the parameters come back unchanged
    p = torch.empty(15601, dtype=torch.float32, device="cuda")
    ctx.guess_get_params(p)
    assert np.array_equal(host(p), flat_params(params).astype(np.float32))


def test_net_gradients_match_oracle():
    n = 10
    ctx, m = lattice_ctx(n, n, n)
    params, x = seeded_net(3, (n, n, n))
    rng = np.random.default_rng(9)
    target = rng.standard_normal((n, n, n)).astype(np.float32).astype(np.float64)
    ctx.guess_set_params(dev(flat_params(params), torch.float32))
    g = torch.empty(15601, dtype=torch.float32, device="cuda")
    loss = ctx.guess_grad(dev(x.reshape(3, -1), torch.float32), dev(target.ravel(), torch.float32), g)
    L, grads = convnet.loss_and_grads(params, x, target)
    assert abs(loss - L) <= 3e-2 * L
    gg = host(g).astype(np.float64)
    off = 0
    for w, b in grads:
        gw = gg[off:off + w.size]
        off += w.size
        gb = gg[off:off + b.size]
        off += b.size
        assert_close(gw, w.ravel(), 3e-2, "weight gradient")
        assert_close(gb, b, 3e-2, "bias gradient")


def test_training_reduces_the_loss():
    n = 12
    ctx, m = lattice_ctx(n, n, n)
    params, x = seeded_net(5, (n, n, n))
    # a target the network can represent: a smooth local function of the inputs
    target = (0.5 * np.tanh(x[0]) - 0.3 * x[1] + 0.1 * x[2]).astype(np.float32)
    ctx.guess_set_params(dev(flat_params(params), torch.float32))
    xi = dev(x.reshape(3, -1), torch.float32)
    ti = dev(target.ravel(), torch.float32)
    first = ctx.guess_train_step(xi, ti, 3e-3)
    for _ in range(300):
        last = ctx.guess_train_step(xi, ti, 3e-3)
    assert last < 0.1 * first, (first, last)


def test_forward_from_initial_guess():
    G = GpuProblem("T12")
    phi, _, info0 = G.forward()
    phi0 = phi.clone().reshape(-1)
    # starting at the solution: converged before any iteration, same answer
    out = torch.empty_like(phi0)
    info = G.ctx.forward_x0(G.kappa, G.mu, phi0, out)
    assert info["iters_max"] <= 1
    assert_close(host(out), host(phi0), 1e-9, "start at the solution")
    # a perturbed start converges to the same tolerance with fewer iterations
    pert = phi0 * (1.0 + 0.01 * torch.sin(torch.arange(phi0.numel(), device="cuda", dtype=torch.float64)))
    info2 = G.ctx.forward_x0(G.kappa, G.mu, pert, out)
    assert info2["relres_max"] <= 1e-10
    assert info2["iters_max"] < info0["iters_max"]
    assert_close(host(out), host(phi0), 1e-8, "start near the solution")
    # a zero start is the plain solve
    info3 = G.ctx.forward_x0(G.kappa, G.mu, torch.zeros_like(phi0), out)
    assert info3["iters_max"] == info0["iters_max"]


def test_trained_guess_saves_pcg_iterations():
    """Train on solver-generated samples of a 24^3 workload (6 Gaussian
    illuminations), evaluate on held-out phantoms: the network's start needs
    fewer PCG iterations than the zero start at the same tolerance."""
    from paper_1512_02796_amd import qpat, learned
    from qpat_inputs import make_problem, initial_params
    P = make_problem("T24")
    m = P.mesh
    ctx = qpat.Context(dev(m.coords), dev(m.tets, torch.int32), dev(m.bfaces, torch.int32))
    ctx.set_sources(dev(P.phi_src))
    n1 = m.n + 1
    ctx.guess_setup(n1, n1, n1)
    ctx.guess_set_params(dev(initial_params(P.cfg["id"]), torch.float32))
    phi_hom = learned.homogeneous_fluence(ctx, P.kappa0, P.mu0, "cuda")
    train = learned.make_samples(ctx, m, 10, P.cfg["id"], 3, "cuda")
    held = learned.make_samples(ctx, m, 3, P.cfg["id"], 4, "cuda")
    hist = learned.train(ctx, train, phi_hom, P.kappa0, P.mu0, epochs=4, lr=2e-3)
    assert hist[-1] < hist[0]
    agg, _ = learned.evaluate(ctx, held, phi_hom, P.kappa0, P.mu0, "cuda")
    assert agg["relres"] <= 1e-10
    assert agg["net_iters"] < agg["zero_iters"], agg
