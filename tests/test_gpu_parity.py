"""HIP path vs the FP64 oracle, element by element, on seeded inputs.

Tolerances. The oracle solves with a sparse LU factorisation (M_delta with
its delta-eigenvector taken exactly); the library with PCG stopped on the
true residual. A PCG solve stopped at rtol has ||x - x*|| / ||x*|| of about
2-3 rtol on these meshes (measured with the oracle's own CG), so the parity
runs use pcg_rtol = prior_rtol = 1e-12 and assert 1e-10 (FP64) element by
element: |a - b| <= 1e-10 (|b| + max|b|). Mixed precision (FP32 operator and
vectors in the Jacobi-PCG K solves, pcg_precond = 0) stops on the same FP64
true residual and is asserted at 1e-6.
"""
import numpy as np
import pytest
import torch

from gpu_util import GpuProblem, oracle_of, data_of, dev, host, rel, need_gpu, assert_close
from qpat_inputs import probe_vectors, kuhn_mesh, make_problem
from oracle import prior as oprior
from oracle.solve import Direct
from oracle.plsqr import PLSQR

pytestmark = pytest.mark.gpu

TIGHT = dict(pcg_rtol=1e-12, prior_rtol=1e-12)


def opts(**kw):
    from paper_1512_02796_amd import qpat
    o = dict(TIGHT)
    o.update(kw)
    return qpat.default_opts(**o)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


# (mesh, block, precision): precision 1 runs the mixed Jacobi-PCG (pcg_precond = 0);
# FP64 runs the default multigrid path. T24 (spacing 40/24 mm, not exact in binary)
# keeps the per-tetrahedron geometry rows, with blocks of 8 right-hand sides.
@pytest.mark.parametrize("name,block,precision", [("T8", 16, 0), ("T12", 1, 0), ("T12", 4, 0), ("T24", 8, 0),
                                                  ("T4", 2, 1), ("T8", 16, 1), ("T24", 8, 1)])
def test_forward_parity(name, block, precision):
    G = GpuProblem(name, opts(max_rhs_block=block, precision=precision, pcg_precond=1 - precision))
    phi, h, info = G.forward()
    g, lin = oracle_of(G.P)
    tol = 1e-10 if precision == 0 else 1e-6
    assert_close(host(phi), lin.phi, tol, f"phi {name}")
    assert_close(host(h), lin.h, tol, f"h {name}")
    assert info["relres_max"] <= 1e-12
    assert info["n_solves"] >= G.n_ill


def test_direction_ring_past_its_length():
    """The tiled K iterations keep their directions and alphas (a ring of 16)
    and form x from them before the true residual; a solve longer than the ring
    forms x in the middle of the run as well. pcg_rtol 1e-14 takes T24 (blocks
    of 8, tiled) past 16 iterations: the result matches the oracle, and the
    same solve run again is bitwise the same."""
    G = GpuProblem("T24", opts(max_rhs_block=8, pcg_rtol=1e-14))
    phi, h, info = G.forward()
    assert info["iters_max"] > 16, info["iters_max"]
    assert info["relres_max"] <= 1e-14
    g, lin = oracle_of(G.P)
    assert_close(host(phi), lin.phi, 1e-10, "phi T24, rtol 1e-14")
    phi2, _, _ = G.forward()
    assert torch.equal(phi, phi2)


def test_restart_from_the_true_residual():
    """At pcg_rtol 5e-16, next to the attainable accuracy, the recursion's
    residual passes the tolerance before the true residual does: the FP64
    true-residual check reopens lanes, which restart from the true residual
    (on the tiled path the check stores no r; it is formed again for the
    restart). The solve still reaches the tolerance and matches the oracle.
    The tile schedule is the cost model's (no timing), so the rounding that
    decides the restarts does not depend on the box (every solve restarts once
    from 3e-16 to 6e-16)."""
    G = GpuProblem("T24", opts(max_rhs_block=8, pcg_rtol=5e-16, autotune=0))
    phi, h, info = G.forward()
    assert info["updates"] > 0, info
    assert info["relres_max"] <= 5e-16, info
    g, lin = oracle_of(G.P)
    assert_close(host(phi), lin.phi, 1e-10, "phi T24, rtol 5e-16")


def test_zero_direction_on_the_tiled_path():
    """J 0 = 0 exactly on the tiled K path (T24, blocks of 8): every tangent
    right-hand side is zero, so each lane stops before iterating and x is
    formed from no directions at all."""
    G = GpuProblem("T24", opts(max_rhs_block=8))
    G.forward()
    out = torch.full((G.n_ill * G.N,), 7.0, dtype=torch.float64, device="cuda")
    info = G.ctx.jvp(torch.zeros(2 * G.N, dtype=torch.float64, device="cuda"), out)
    assert torch.count_nonzero(out).item() == 0
    assert info["iters_max"] == 0


@pytest.mark.parametrize("name,block,precision", [("T8", 4, 0), ("T12", 1, 0), ("T24", 8, 0),
                                                  ("T12", 4, 1), ("T24", 8, 1)])
def test_jvp_vjp_parity(name, block, precision):
    G = GpuProblem(name, opts(max_rhs_block=block, precision=precision, pcg_precond=1 - precision))
    if name == "T24":
        assert G.ctx.geometry_classes() == 0          # the per-tetrahedron rows run
    G.forward()
    g, lin = oracle_of(G.P)
    s, t = probe_vectors(G.P.cfg["id"], G.n_ill, G.N)
    out = torch.empty(G.n_ill * G.N, dtype=torch.float64, device="cuda")
    G.ctx.jvp(dev(s), out)
    tol = 1e-10 if precision == 0 else 1e-6
    assert_close(host(out).reshape(G.n_ill, G.N), lin.jvp(s), tol, f"J s {name}")
    outT = torch.empty(2 * G.N, dtype=torch.float64, device="cuda")
    G.ctx.vjp(dev(t), outT)
    assert_close(host(outT), lin.vjp(t), tol, f"J^T t {name}")


@pytest.mark.parametrize("name,n_ill", [("T8", 16), ("T12", 9)])
def test_mixed_multigrid_parity(name, n_ill):
    """precision = 1 on the multigrid path: with 16 right-hand sides on the tiled
    kernels (9 or 16 illuminations: one block of 16) the direction p is stored in
    FP32 while x, r, q = A p and the dots stay FP64, so the solves meet the same
    FP64 true-residual rule and the products match the oracle at the FP64
    tolerance."""
    G = GpuProblem(name, opts(max_rhs_block=16, precision=1), n_ill=n_ill)
    phi, h, info = G.forward()
    g, lin = oracle_of(G.P)
    assert info["relres_max"] <= 1e-12
    assert_close(host(phi), lin.phi, 1e-10, f"phi {name} mixed multigrid")
    s, t = probe_vectors(G.P.cfg["id"], G.n_ill, G.N)
    out = torch.empty(G.n_ill * G.N, dtype=torch.float64, device="cuda")
    G.ctx.jvp(dev(s), out)
    assert_close(host(out).reshape(G.n_ill, G.N), lin.jvp(s), 1e-10, f"J s {name} mixed multigrid")
    outT = torch.empty(2 * G.N, dtype=torch.float64, device="cuda")
    G.ctx.vjp(dev(t), outT)
    assert_close(host(outT), lin.vjp(t), 1e-10, f"J^T t {name} mixed multigrid")


def test_per_rhs_report():
    """qpat_info's per-system arrays: one entry per right-hand side solved (the
    padding columns of the last block included), consistent with the aggregates."""
    G = GpuProblem("T24", opts(max_rhs_block=4))       # 6 illuminations -> blocks of 4 and 4 (2 padded)
    phi, h, info = G.forward()
    it, rr = info["rhs_iters"], info["rhs_relres"]
    assert info["n_solves"] == len(it) == len(rr) == 8
    assert max(it) == info["iters_max"] and sum(it) == info["iters_sum"]
    assert max(rr) == info["relres_max"] and all(r <= 1e-12 for r in rr)
    assert it[6] == 0 and it[7] == 0 and rr[6] == 0.0 and rr[7] == 0.0   # zero right-hand sides
    assert all(i > 0 for i in it[:6])


def test_init_guess_averages_over_illuminations():
    """qpat_init_guess on data chi_k = c_k mu0 phi0_k with distinct c_k: mt_init =
    log(mean_k c_k) at every node (the average of exp(mt_init^(k)), Sec. 4 after
    Algorithm 1; a geometric mean would give log(sqrt 2)), kt_init = 0."""
    P = make_problem("T8")
    G = GpuProblem("T8", opts())
    N = G.N
    beta = torch.zeros(2 * N, dtype=torch.float64, device="cuda")
    G.ctx.forward_log(P.kappa0, P.mu0, beta)
    phi0 = torch.empty(G.n_ill * N, dtype=torch.float64, device="cuda")
    G.ctx.forward(dev(np.full(N, P.kappa0)), dev(np.full(N, P.mu0)), phi0)
    c = np.array([0.5, 1.0, 2.0, 4.0])
    chi = c[:, None] * P.mu0 * host(phi0).reshape(G.n_ill, N)
    out = torch.full((2 * N,), 3.0, dtype=torch.float64, device="cuda")
    G.ctx.init_guess(dev(chi), P.mu0, out)
    r = host(out)
    assert np.all(r[:N] == 0.0)
    # the oracle's initial_guess gives log(mean c_k) on the same data (pinned on
    # the CPU); a comparison through the oracle's own fluence would only measure
    # the two solves' pointwise relative error at nodes of tiny fluence
    assert np.abs(r[N:] - np.log(1.875)).max() <= 1e-14


def test_adjoint_identity_on_gpu():
    G = GpuProblem("T12", opts(pcg_rtol=1e-13))
    G.forward()
    s, t = probe_vectors(G.P.cfg["id"], G.n_ill, G.N)
    Js = torch.empty(G.n_ill * G.N, dtype=torch.float64, device="cuda")
    Jt = torch.empty(2 * G.N, dtype=torch.float64, device="cuda")
    G.ctx.jvp(dev(s), Js)
    G.ctx.vjp(dev(t), Jt)
    lhs = float(torch.dot(Js, dev(t).reshape(-1)))
    rhs = float(torch.dot(dev(s), Jt))
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), abs(rhs))


@pytest.mark.parametrize("deflate,rtol,tol", [(1, 1e-12, 1e-10), (0, 2e-10, 1e-7)])
def test_prior_apply_and_solve(deflate, rtol, tol):
    """M_delta and M_delta^{-1} against the oracle's, whose inverse takes the
    delta-eigenvector (mean(p)/delta per block) exactly. With deflation the
    library solves the same split and meets 1e-10 element by element at
    prior_rtol 1e-12; without it the delta-eigenvector (|x| ~ mean/delta) limits
    FP64 PCG to a true residual near 1e-10 (eps cond(M_delta)), hence 1e-7."""
    G = GpuProblem("T12", opts(prior_deflate=deflate, prior_rtol=rtol))
    P = G.P
    kt = np.log(P.kappa / P.kappa0)
    mt = np.log(P.mu / P.mu0)
    G.ctx.prior_setup(dev(kt), dev(mt), 5e-3, 1.7, 1e-6)
    g, _ = oracle_of(P)
    Pr = oprior.Prior(g, kt, mt, 5e-3, 1.7, 1e-6, solver="deflated")
    rng = np.random.default_rng(11)
    x = rng.standard_normal(2 * G.N)
    y = torch.empty(2 * G.N, dtype=torch.float64, device="cuda")
    G.ctx.prior_apply(dev(x), y)
    assert_close(host(y), Pr.apply(x), 1e-14, "M_delta x")
    r = torch.empty_like(y)
    info = G.ctx.prior_solve(dev(x), r)
    assert info["relres_max"] <= rtol, info
    assert_close(host(r), Pr.solve(x), tol, "M_delta^-1 p")


@pytest.mark.parametrize("q,precond", [(1.0, 1), (0.5, 1), (1.5, 0)])
def test_prior_tvq_apply_and_solve(q, precond):
    """TV^q prior (r(t) = T^(2-q) (t^2 + T^2)^(q/2) / q): the library's M_delta and
    M_delta^{-1} against the oracle's (exact delta-eigenvector), multigrid and
    Jacobi preconditioners, element by element at 1e-10."""
    from paper_1512_02796_amd import qpat
    G = GpuProblem("T12", opts(prior_precond=precond, prior_rtol=1e-12))
    P = G.P
    kt = np.log(P.kappa / P.kappa0)
    mt = np.log(P.mu / P.mu0)
    G.ctx.prior_setup_r(dev(kt), dev(mt), qpat.PRIOR_TVQ, 5e-3, q, 1.7, 1e-6)
    g, _ = oracle_of(P)
    Pr = oprior.Prior(g, kt, mt, 5e-3, 1.7, 1e-6, solver="deflated", kind="tvq", q=q)
    rng = np.random.default_rng(12)
    x = rng.standard_normal(2 * G.N)
    y = torch.empty(2 * G.N, dtype=torch.float64, device="cuda")
    G.ctx.prior_apply(dev(x), y)
    assert_close(host(y), Pr.apply(x), 1e-14, "M_delta x")
    r = torch.empty_like(y)
    info = G.ctx.prior_solve(dev(x), r)
    assert info["relres_max"] <= 1e-12, info
    assert_close(host(r), Pr.solve(x), 1e-10, "M_delta^-1 p")


def test_graph_cache_tracks_the_region_count():
    """One context, two prior set-ups whose region coarse spaces differ in size
    (a constant field: one region, dropped under deflation; the phantom: several):
    the second M_delta^{-1} replays no graph captured for the first, so result and
    iteration count equal those of a fresh context without graphs."""
    P = make_problem("T24")
    kt = np.log(P.kappa / P.kappa0)
    mt = np.log(P.mu / P.mu0)
    p = np.random.default_rng(21).standard_normal(2 * P.mesh.N)
    zero = np.zeros(P.mesh.N)
    outs, infos = [], []
    for graphs, setups in ((1, [(zero, zero), (kt, mt)]), (0, [(kt, mt)])):
        G = GpuProblem("T24", opts(use_graphs=graphs, prior_rtol=1e-10))
        for a, b in setups:
            G.ctx.prior_setup(dev(a), dev(b))
            out = torch.empty(2 * P.mesh.N, dtype=torch.float64, device="cuda")
            info = G.ctx.prior_solve(dev(p), out)
        outs.append(host(out))
        infos.append(info)
    assert infos[0]["rhs_iters"] == infos[1]["rhs_iters"], infos
    assert np.array_equal(outs[0], outs[1])


def test_prior_setup_r_rejects_bad_arguments():
    from paper_1512_02796_amd import qpat
    G = GpuProblem("T4")
    z = torch.zeros(G.N, dtype=torch.float64, device="cuda")
    for kind, q in ((qpat.PRIOR_TVQ, 0.0), (qpat.PRIOR_TVQ, 2.5), (7, 1.0)):
        with pytest.raises(qpat.QpatError) as e:
            G.ctx.prior_setup_r(z, z, kind, 5e-3, q)
        assert "ERR_ARG" in str(e.value)
    G.ctx.prior_setup_r(z, z, qpat.PRIOR_PM, 5e-3, -1.0)   # q is ignored for Perona-Malik


def _oracle_plsqr(G, W, chi, steps, reorth=True):
    P = G.P
    g, lin = oracle_of(P)
    kt = np.log(P.kappa / P.kappa0)
    mt = np.log(P.mu / P.mu0)
    beta_lin = np.concatenate([kt, mt])
    Pr = oprior.Prior(g, kt, mt, solver="deflated")
    n_ill, N = P.n_ill, G.N
    yt = (W * (chi - lin.h + lin.jvp(beta_lin))).ravel()
    it = PLSQR(lambda v: (W * lin.jvp(v)).ravel(), lambda u: lin.vjp(W * u.reshape(n_ill, N)), Pr.solve, yt,
               reorth=reorth)
    for _ in range(steps):
        it.step()
    return it, beta_lin


@pytest.mark.parametrize("whiten,hist_tol,x_tol", [("const", 1e-10, 1e-10), ("noise", 1e-8, 1e-8)])
def test_lsqr_matches_oracle(whiten, hist_tol, x_tol):
    """8 PLSQR steps from the same chi and W, against the oracle's PLSQR with the
    exact-deflation M_delta^{-1}. With W = 1/(sigma |h|) (the data model) W
    amplifies the pointwise error of h at nodes of tiny fluence, which the K
    solves (pcg_rtol 1e-13 here) bound only in norm."""
    G = GpuProblem("T8", opts(pcg_rtol=1e-13))
    G.forward()
    P = G.P
    g, lin = oracle_of(P)
    chi, W = data_of(P, lin)
    if whiten == "const":
        W = np.full_like(W, 1.0 / (P.cfg["noise"] * np.abs(lin.h).mean()))
    steps = 8
    it, beta_lin = _oracle_plsqr(G, W, chi, steps)
    kt, mt = beta_lin[:G.N], beta_lin[G.N:]
    G.ctx.prior_setup(dev(kt), dev(mt))
    x = torch.zeros(2 * G.N, dtype=torch.float64, device="cuda")
    G.ctx.lsqr_init(dev(chi), dev(W), dev(beta_lin), x)
    hist = [G.ctx.lsqr_residual()]
    for _ in range(steps):
        res, _ = G.ctx.lsqr_step()
        hist.append(res)
    assert_close(np.array(hist), np.array(it.history), hist_tol, "LSQR residual history")
    assert_close(host(x), it.x, x_tol, "LSQR iterate")
    assert G.ctx.lsqr_steps() == steps


def test_lsqr_runs_past_the_initial_basis_capacity():
    """lsqr_max_steps = 3: the reorthogonalised run fills its bases after 3 steps
    and grows them; 9 steps match the oracle's fully reorthogonalised PLSQR."""
    G = GpuProblem("T8", opts(pcg_rtol=1e-13, lsqr_max_steps=3))
    G.forward()
    P = G.P
    g, lin = oracle_of(P)
    chi, W = data_of(P, lin)
    W = np.full_like(W, 1.0 / (P.cfg["noise"] * np.abs(lin.h).mean()))
    steps = 9
    it, beta_lin = _oracle_plsqr(G, W, chi, steps)
    G.ctx.prior_setup(dev(beta_lin[:G.N]), dev(beta_lin[G.N:]))
    x = torch.zeros(2 * G.N, dtype=torch.float64, device="cuda")
    G.ctx.lsqr_init(dev(chi), dev(W), dev(beta_lin), x)
    hist = [G.ctx.lsqr_residual()]
    for _ in range(steps):
        hist.append(G.ctx.lsqr_step()[0])
    assert G.ctx.lsqr_basis() == steps + 1
    assert_close(np.array(hist), np.array(it.history), 1e-10, "LSQR residual history")
    assert_close(host(x), it.x, 1e-10, "LSQR iterate")


def test_block_sizes_agree_and_deterministic():
    outs = []
    for block in (1, 2, 16):
        G = GpuProblem("T8", opts(max_rhs_block=block))
        phi, _, _ = G.forward()
        outs.append(host(phi))
    assert_close(outs[0], outs[2], 1e-11, "block 1 vs 16")
    assert_close(outs[1], outs[2], 1e-11, "block 2 vs 16")
    G = GpuProblem("T8", opts())
    a, _, _ = G.forward()
    a = host(a).copy()
    b, _, _ = G.forward()
    assert np.array_equal(a, host(b))


def test_error_paths():
    from paper_1512_02796_amd import qpat
    m = kuhn_mesh(2, 40.0)
    bad = m.tets.copy()
    bad[3, 2] = m.N + 5
    with pytest.raises(qpat.QpatError) as e:
        qpat.Context(dev(m.coords), dev(bad, torch.int32), dev(m.bfaces, torch.int32))
    assert e.value.status == qpat.QPAT_ERR_MESH
    flat = m.coords.copy()
    flat[:, 2] = 0.0
    with pytest.raises(qpat.QpatError) as e:
        qpat.Context(dev(flat), dev(m.tets, torch.int32), dev(m.bfaces, torch.int32))
    assert e.value.status == qpat.QPAT_ERR_MESH
    ctx = qpat.Context(dev(m.coords), dev(m.tets, torch.int32), dev(m.bfaces, torch.int32))
    ctx.set_sources(dev(np.ones((1, m.F_b, 3))))
    s = torch.zeros(2 * m.N, dtype=torch.float64, device="cuda")
    out = torch.zeros(m.N, dtype=torch.float64, device="cuda")
    with pytest.raises(qpat.QpatError) as e:       # J before any forward solve
        ctx.jvp(s, out)
    assert e.value.status == qpat.QPAT_ERR_STATE
    with pytest.raises(qpat.QpatError) as e:       # prior solve before prior setup
        ctx.prior_solve(s, torch.zeros_like(s))
    assert e.value.status == qpat.QPAT_ERR_STATE
    kap = torch.full((m.N,), 0.3, dtype=torch.float64, device="cuda")
    mu = torch.full((m.N,), -0.01, dtype=torch.float64, device="cuda")
    with pytest.raises(qpat.QpatError) as e:
        ctx.forward(kap, mu)
    assert e.value.status == qpat.QPAT_ERR_ARG
    mu.fill_(0.01)
    ctx.set_opts(pcg_maxit=1)
    with pytest.raises(qpat.QpatError) as e:
        ctx.forward(kap, mu)
    assert e.value.status == qpat.QPAT_ERR_NOCONV


def test_graph_replays_match_eager():
    """Chunks of PCG iterations replayed as captured HIP graphs give the eager
    launches' result bit for bit, replay after replay, with eager work between."""
    G = GpuProblem("T12", opts(use_graphs=0))
    a, _, _ = G.forward()
    a = host(a).copy()
    for _ in range(3):
        G.ctx.set_opts(use_graphs=1)
        b, _, _ = G.forward()
        assert np.array_equal(a, host(b))
        G.ctx.set_opts(use_graphs=0)
        c, _, _ = G.forward()
        assert np.array_equal(a, host(c))


def test_geometry_classes_on_an_exact_lattice():
    """8^3 voxels on 40 mm (spacing 5, exact): the 6 Kuhn tetrahedron shapes are the
    classes, and the forward/J products through them match the oracle (the other
    parity tests run meshes with inexact spacings through the per-tetrahedron rows)."""
    G = GpuProblem("T8", opts())
    assert G.ctx.geometry_classes() == 6
    G.forward()
    g, lin = oracle_of(G.P)
    s, t = probe_vectors(G.P.cfg["id"], G.n_ill, G.N)
    out = torch.empty(G.n_ill * G.N, dtype=torch.float64, device="cuda")
    G.ctx.jvp(dev(s), out)
    assert_close(host(out).reshape(G.n_ill, G.N), lin.jvp(s), 1e-10, "J s")
    outT = torch.empty(2 * G.N, dtype=torch.float64, device="cuda")
    G.ctx.vjp(dev(t), outT)
    assert_close(host(outT), lin.vjp(t), 1e-10, "J^T t")
    H = GpuProblem("T12", opts())
    assert H.ctx.geometry_classes() in (0, 6)


def test_autotuned_tile_schedule():
    """opts.autotune times the cost model's lowest-cost z-chunk lengths of the tiled
    kernels at the first solve and keeps the fastest: the schedule reports a tuned
    length among those candidates, and the forward fluence equals the untuned
    context's up to the order of the partial sums."""
    P = dict(n_ill=16)
    G0 = GpuProblem("T12", opts(max_rhs_block=16, autotune=0), **P)
    G1 = GpuProblem("T12", opts(max_rhs_block=16, autotune=1), **P)
    phi0, _, _ = G0.forward()
    phi1, _, _ = G1.forward()
    s0, s1 = G0.ctx.tile_schedule(16), G1.ctx.tile_schedule(16)
    assert s0["tiled"] and s1["tiled"] and not s0["tuned"] and s1["tuned"]
    assert s0["zc"] == s0["zc_model"] and s1["zc_model"] == s0["zc_model"]
    nz = G1.ctx.operator_layout()["nz"]
    assert 1 <= s1["zc"] <= nz and s1["ps_zc"] % 2 == 0 and s1["ps_zc32"] % 2 == 0
    assert_close(host(phi1), host(phi0), 1e-12, "phi tuned vs untuned")
