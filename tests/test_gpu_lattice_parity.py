"""Parity on lattices large enough for the multigrid's tiled coarse levels.

The 16-right-hand-side K solves run the finest level LDS-tiled and, on every
coarse level of at least 16384 nodes, the tiled 27-point residual and sweep
kernels (and the tiled restriction into such a level). A 128 x 128 x 8 voxel
slab has 129 x 129 x 9 nodes and a first coarse level of 65 x 65 x 5 = 21125
nodes, so its level 1 runs tiled; the slab keeps the oracle's sparse LU cheap
(its separators are 9 planes thick). The spacing 0.3 mm is not exact in
binary, so the Jacobian's element kernels read the per-tetrahedron geometry
rows. 16 illuminations with random vertex values of Phi on every boundary
triangle, random log-normal kappa and mu.

Checked element by element, |a - b| <= 1e-10 (|b| + max|b|), against the FP64
oracle (sparse LU): fluence, J s and J^T t.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, need_gpu, assert_close
from test_gpu_stencil import box_problem
from oracle import fem
from oracle.jacobian import Linearisation

pytestmark = pytest.mark.gpu

DIMS, N_ILL, SPACING = (128, 128, 8), 16, 0.3


def coarse(n):
    return n // 2 + 1 if n > 2 else n


@pytest.fixture(scope="module")
def slab():
    need_gpu()
    from paper_1512_02796_amd import qpat
    coords, tets, bfaces, kappa, mu, src = box_problem(*DIMS, N_ILL, seed=1512)
    coords = coords * SPACING
    nx, ny, nz = (d + 1 for d in DIMS)
    assert coarse(nx) * coarse(ny) * coarse(nz) >= 16384          # level 1 runs tiled
    print(f"slab {DIMS}: N = {coords.shape[0]}, oracle factorisation ...", flush=True)
    g = fem.geometry(coords, tets, bfaces)
    lin = Linearisation(g, kappa, mu, src, solver="direct_sym")
    rng = np.random.default_rng(15)
    s = rng.standard_normal(2 * coords.shape[0])
    t = rng.standard_normal((N_ILL, coords.shape[0]))
    ctx = qpat.Context(dev(coords), dev(tets, torch.int32), dev(bfaces, torch.int32),
                       opts=qpat.default_opts(pcg_rtol=1e-12, max_rhs_block=16))
    ctx.set_sources(dev(src))
    yield dict(ctx=ctx, lin=lin, kappa=kappa, mu=mu, s=s, t=t, N=coords.shape[0])
    ctx.close()


def test_slab_uses_the_lattice_path(slab):
    lay = slab["ctx"].operator_layout()
    assert lay["lattice"] and (lay["nx"], lay["ny"], lay["nz"]) == tuple(d + 1 for d in DIMS)
    assert slab["ctx"].geometry_classes() == 0


def test_slab_forward_parity(slab):
    ctx, lin, N = slab["ctx"], slab["lin"], slab["N"]
    phi = torch.empty(N_ILL * N, dtype=torch.float64, device="cuda")
    info = ctx.forward(dev(slab["kappa"]), dev(slab["mu"]), phi)
    assert info["relres_max"] <= 1e-12 and info["n_solves"] == N_ILL
    assert_close(host(phi).reshape(N_ILL, N), lin.phi, 1e-10, "slab fluence")


def test_slab_jvp_vjp_parity(slab):
    ctx, lin, N = slab["ctx"], slab["lin"], slab["N"]
    ctx.forward(dev(slab["kappa"]), dev(slab["mu"]))
    out = torch.empty(N_ILL * N, dtype=torch.float64, device="cuda")
    ctx.jvp(dev(slab["s"]), out)
    assert_close(host(out).reshape(N_ILL, N), lin.jvp(slab["s"]), 1e-10, "slab J s")
    outT = torch.empty(2 * N, dtype=torch.float64, device="cuda")
    ctx.vjp(dev(slab["t"]), outT)
    assert_close(host(outT), lin.vjp(slab["t"]), 1e-10, "slab J^T t")


def test_slab_mixed_precision_parity(slab):
    """The same products with precision = 1: the tiled 16-right-hand-side path
    stores the PCG direction in FP32 (x, r, q = A p and the dots in FP64), so the
    FP64 tolerance still holds."""
    ctx, lin, N = slab["ctx"], slab["lin"], slab["N"]
    ctx.set_opts(precision=1)
    try:
        phi = torch.empty(N_ILL * N, dtype=torch.float64, device="cuda")
        info = ctx.forward(dev(slab["kappa"]), dev(slab["mu"]), phi)
        assert info["relres_max"] <= 1e-12
        assert_close(host(phi).reshape(N_ILL, N), lin.phi, 1e-10, "slab fluence, mixed")
        out = torch.empty(N_ILL * N, dtype=torch.float64, device="cuda")
        ctx.jvp(dev(slab["s"]), out)
        assert_close(host(out).reshape(N_ILL, N), lin.jvp(slab["s"]), 1e-10, "slab J s, mixed")
        outT = torch.empty(2 * N, dtype=torch.float64, device="cuda")
        ctx.vjp(dev(slab["t"]), outT)
        assert_close(host(outT), lin.vjp(slab["t"]), 1e-10, "slab J^T t, mixed")
    finally:
        ctx.set_opts(precision=0)


def test_graded_lattice_products():
    """A lattice numbering with unequal voxels (x graded): the stencil form still
    applies, the voxel form of the G kernels (equal voxels only) must be turned
    down by its set-up comparison with the element form, and J s, J^T t match
    the oracle at the FP64 tolerance through 16-right-hand-side blocks."""
    from paper_1512_02796_amd import qpat
    from qpat_inputs import make_problem, probe_vectors
    from gpu_util import assert_close, dev, host, oracle_of
    P = make_problem("T8", n_ill=16)
    m = P.mesh
    L = float(m.coords[:, 0].max())
    m.coords[:, 0] = L * (m.coords[:, 0] / L) ** 1.25   # monotone: the numbering stays lexicographic
    ctx = qpat.Context(dev(m.coords), dev(m.tets, torch.int32), dev(m.bfaces, torch.int32),
                       opts=qpat.default_opts(max_rhs_block=16))
    ctx.set_sources(dev(P.phi_src))
    phi = torch.empty(P.n_ill * m.N, dtype=torch.float64, device="cuda")
    h = torch.empty_like(phi)
    ctx.forward(dev(P.kappa), dev(P.mu), phi, h)
    g, lin = oracle_of(P)
    assert_close(host(phi).reshape(P.n_ill, m.N), lin.phi, 1e-10, "phi graded")
    s, t = probe_vectors(P.cfg["id"], P.n_ill, m.N)
    out = torch.empty(P.n_ill * m.N, dtype=torch.float64, device="cuda")
    ctx.jvp(dev(s), out)
    assert_close(host(out).reshape(P.n_ill, m.N), lin.jvp(s), 1e-10, "J s graded lattice")
    outT = torch.empty(2 * m.N, dtype=torch.float64, device="cuda")
    ctx.vjp(dev(t), outT)
    assert_close(host(outT), lin.vjp(t), 1e-10, "J^T t graded lattice")
