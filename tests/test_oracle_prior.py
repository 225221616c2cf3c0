"""Pins of the oracle's lagged-diffusivity priors (Perona-Malik and TV^q)."""
import numpy as np
import pytest

from qpat_inputs import kuhn_mesh, make_problem
from oracle import fem, prior
from oracle.solve import Direct, pcg

T = 5e-3


def geo(n=4):
    m = kuhn_mesh(n, 40.0)
    return m, fem.geometry(m.coords, m.tets, m.bfaces)


def test_diffusivity_is_derivative_ratio():
    """c(t) = r'(t)/t with r(t) = (T^2/2) log(1 + (t/T)^2): check r' by central differences."""
    def r(t):
        return 0.5 * T * T * np.log1p((t / T) ** 2)
    t = np.array([1e-4, 3e-3, 5e-3, 0.02, 0.7])
    d = 1e-7 * t
    fd = (r(t + d) - r(t - d)) / (2 * d)
    assert np.allclose(prior.r_prime(t, T), fd, rtol=1e-7)
    assert np.allclose(prior.diffusivity(t, T), fd / t, rtol=1e-7)
    assert prior.diffusivity(np.array([0.0]), T)[0] == 1.0


def test_M_kernel_and_semidefinite():
    P = make_problem("T8")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    u = np.log(P.kappa / P.kappa0)
    M = prior.M_of(g, u, T)
    one = np.ones(g.N)
    assert np.abs(M @ one).max() < 1e-13 * np.abs(M).max()
    assert abs(M - M.T).max() <= 1e-15 * abs(M).max()
    rng = np.random.default_rng(0)
    for _ in range(5):
        v = rng.standard_normal(g.N)
        assert v @ (M @ v) >= 0.0
    ev = np.linalg.eigvalsh(M.toarray())
    assert ev[0] > -1e-12 * ev[-1] and ev[1] > 1e-10 * ev[-1]      # Ker M = span{1}


def test_constant_u_gives_laplacian():
    m, g = geo(3)
    M = prior.M_of(g, np.full(m.N, 0.37), T)
    S = fem.stiffness(g, np.ones(m.N))
    assert np.allclose(M.toarray(), S.toarray(), rtol=1e-13, atol=1e-15)


def test_linear_u_scales_laplacian():
    """u = g.x has |grad u| = |g| everywhere, so M = S(1) / (1 + |g|^2 / T^2)."""
    m, g = geo(3)
    gvec = np.array([2e-3, -4e-3, 1e-3])
    M = prior.M_of(g, m.coords @ gvec, T)
    S = fem.stiffness(g, np.ones(m.N))
    want = S / (1 + (gvec @ gvec) / T ** 2)
    assert np.allclose(M.toarray(), want.toarray(), rtol=1e-12, atol=1e-15)


def test_M_delta_structure():
    P = make_problem("T4")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    kt = np.log(P.kappa / P.kappa0)
    mt = np.log(P.mu / P.mu0)
    N = g.N
    Md = prior.M_delta(g, kt, mt, T, b_over_a=2.5, delta=1e-6).toarray()
    Mk = prior.M_of(g, kt, T).toarray()
    Mm = prior.M_of(g, mt, T).toarray()
    assert np.allclose(Md[:N, :N], Mk + 1e-6 * np.eye(N), rtol=1e-14, atol=1e-20)
    assert np.allclose(Md[N:, N:], 2.5 * Mm + 1e-6 * np.eye(N), rtol=1e-14, atol=1e-20)
    assert np.all(Md[:N, N:] == 0) and np.all(Md[N:, :N] == 0)
    # the constant vectors are eigenvectors with eigenvalue delta
    e = np.concatenate([np.ones(N), np.zeros(N)])
    assert np.allclose(Md @ e, 1e-6 * e, atol=1e-15)


def test_M_delta_solve_direct_vs_pcg():
    P = make_problem("T8")
    g = fem.geometry(P.mesh.coords, P.mesh.tets, P.mesh.bfaces)
    kt = np.log(P.kappa / P.kappa0)
    mt = np.log(P.mu / P.mu0)
    Md = prior.M_delta(g, kt, mt)
    rng = np.random.default_rng(1)
    p = rng.standard_normal(2 * g.N)
    xd = Direct(Md)(p)
    info = {}
    xc = pcg(Md, p, rtol=1e-10, info=info)
    assert info["relres"] <= 1e-10
    assert np.linalg.norm(Md @ xd - p) <= 1e-9 * np.linalg.norm(p)   # eps ||M|| ||x||
    # ||dx|| / ||x|| <= cond(M_delta) rtol in the worst case; cond ~ ||M|| / delta
    # is ~1e8 here, but the error along the delta-eigenvector 1 is tiny because
    # its component is fixed by the mean: 1.(M_delta x) = delta 1.x per block
    assert np.linalg.norm(xc - xd) <= 1e-8 * np.linalg.norm(xd)
    N = g.N
    assert abs(1e-6 * xd[:N].sum() - p[:N].sum()) <= 1e-9 * np.abs(p[:N]).sum()
    assert abs(1e-6 * xd[N:].sum() - p[N:].sum()) <= 1e-9 * np.abs(p[N:]).sum()


KINDS = [("pm", 1.0), ("tvq", 1.0), ("tvq", 0.5), ("tvq", 1.5)]


@pytest.mark.parametrize("kind,q", KINDS)
def test_gradient_of_R_is_M_u(kind, q):
    """grad R(u) = M(u) u (Sec. 4, after eq. (4.2)), with R(u) = sum_T |T| r(|grad u_T|)
    evaluated from r alone and differentiated by central differences: this pins
    c = r'(t)/t against r for each choice, independently of how M is formed."""
    m, g = geo(3)
    rng = np.random.default_rng(5)
    u = 0.01 * rng.standard_normal(m.N)   # |grad u| ~ T, where r bends most
    Mu = prior.M_of(g, u, T, kind, q) @ u
    h = 1e-7
    fd = np.empty(m.N)
    for i in range(m.N):
        e = np.zeros(m.N)
        e[i] = h
        fd[i] = (prior.R_of(g, u + e, T, kind, q) - prior.R_of(g, u - e, T, kind, q)) / (2 * h)
    assert np.linalg.norm(fd - Mu) <= 1e-6 * np.linalg.norm(Mu)


@pytest.mark.parametrize("q", [0.5, 1.0, 1.5, 2.0])
def test_tvq_linear_u_closed_form(q):
    """u = g.x: |grad u| = |g| on every tetrahedron, so M = S(1) (1 + |g|^2/T^2)^((q-2)/2);
    q = 2 gives the plain Laplacian stiffness for any u."""
    m, g = geo(3)
    gvec = np.array([2e-3, -4e-3, 1e-3])
    M = prior.M_of(g, m.coords @ gvec, T, "tvq", q)
    S = fem.stiffness(g, np.ones(m.N))
    want = S * (1 + (gvec @ gvec) / T ** 2) ** ((q - 2) / 2)
    assert np.allclose(M.toarray(), want.toarray(), rtol=1e-12, atol=1e-15)
    if q == 2.0:
        rng = np.random.default_rng(3)
        M2 = prior.M_of(g, rng.standard_normal(m.N), T, "tvq", 2.0)
        assert np.allclose(M2.toarray(), S.toarray(), rtol=1e-13, atol=1e-15)


def test_smoothed_tv_limits():
    """q = 1: r(t) = T sqrt(t^2 + T^2), so c(t) -> T/t for t >> T (the TV diffusivity
    1/|grad u| scaled by T), c(0) = 1, and r is increasing (Sec. 3 asks for that)."""
    t = np.array([1e-1, 1.0, 10.0])
    c = prior.diffusivity(t, T, "tvq", 1.0)
    assert np.allclose(c, T / t, rtol=(T / t).max() ** 2)
    assert prior.diffusivity(np.array([0.0]), T, "tvq", 1.0)[0] == 1.0
    tt = np.linspace(0, 0.1, 101)
    for q in (0.5, 1.0, 1.5, 2.0):
        assert np.all(np.diff(prior.r_of(tt, T, "tvq", q)) > 0)


def _exact_solve(A, b, delta):
    """(A0 + delta I) x = b in exact rational arithmetic, where A0 has the
    off-diagonal entries of A (exact binary rationals) and the diagonal that
    makes every row sum to zero exactly -- the kernel property M(u) 1 = 0 that
    the floating-point assembly holds only to rounding. Gaussian elimination
    over Fractions, rounded once at the end."""
    from fractions import Fraction
    n = A.shape[0]
    M = [[Fraction(float(A[i, j])) if i != j else Fraction(0) for j in range(n)] for i in range(n)]
    for i in range(n):
        M[i][i] = -sum(M[i]) + Fraction(delta)
        M[i].append(Fraction(float(b[i])))
    for k in range(n):
        piv = next(i for i in range(k, n) if M[i][k] != 0)
        M[k], M[piv] = M[piv], M[k]
        for i in range(k + 1, n):
            f = M[i][k] / M[k][k]
            if f:
                row_k = M[k]
                M[i] = [a - f * c for a, c in zip(M[i], row_k)]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        s = M[i][n] - sum(M[i][j] * x[j] for j in range(i + 1, n))
        x[i] = s / M[i][i]
    return np.array([float(v) for v in x])


def _ideal_residual(Md, N, x, p, delta):
    """M_delta x - p with each block's rows made to sum to zero exactly: the
    constant part of x (mean/delta, of size ~1/delta) is multiplied by zero
    instead of by the assembly's rounding."""
    out = np.empty(2 * N)
    for j in range(2):
        B = Md[j * N:(j + 1) * N, j * N:(j + 1) * N]
        xj = x[j * N:(j + 1) * N]
        xc = xj - xj.mean()
        rowsum = np.asarray(B.sum(axis=1)).ravel() - delta
        out[j * N:(j + 1) * N] = B @ xc - rowsum * xc + delta * xj.mean() - p[j * N:(j + 1) * N]
    return out


def test_deflated_solve_matches_exact_rational_solve():
    """M_delta^{-1} with the delta-eigenvector taken exactly (mean(p)/delta per
    block, LU on the mean-free rest) equals the exact rational solution of the
    same matrix with M(u) 1 = 0 imposed exactly, to 1e-13 element by element, on
    a 2^3 mesh with jumps of kt and mt that take c_T down to ~1e-2 and
    b/a != 1 (so a swapped block scale or a dropped mean term fails)."""
    m, g = geo(2)
    rng = np.random.default_rng(5)
    kt = np.where(rng.random(g.N) < 0.5, 0.0, 1.0)
    mt = rng.standard_normal(g.N)
    b_over_a, delta = 1.7, 1e-6
    P = prior.Prior(g, kt, mt, T, b_over_a, delta, solver="deflated")
    Md = P.Md.toarray()
    p = rng.standard_normal(2 * g.N) + 0.3
    x = P.solve(p)
    N = g.N
    ref = np.concatenate([_exact_solve(Md[:N, :N], p[:N], delta), _exact_solve(Md[N:, N:], p[N:], delta)])
    assert np.all(np.abs(x - ref) <= 1e-13 * (np.abs(ref) + np.abs(ref).max()))
    # the mean of each block is mean(p)/delta, exactly the delta-eigenvector part
    assert abs(ref[:N].mean() - p[:N].mean() / delta) <= 1e-12 * abs(p[:N].mean() / delta)
    assert abs(ref[N:].mean() - p[N:].mean() / delta) <= 1e-12 * abs(p[N:].mean() / delta)


def test_deflated_solve_is_more_accurate_than_plain_lu():
    """On the 8^3 phantom the deflated solve's residual with rows summing to zero
    exactly stays below 1e-10 -- the floor is the assembly's row sums (~1e-16
    |M_ii|) times the mean-free part of the solution, whose size is set by the
    smallest non-zero eigenvalue of M(u), not by delta -- and each block's mean is
    mean(p)/delta. The plain LU of M_delta agrees only to about eps cond(M_delta)."""
    P8 = make_problem("T8")
    g = fem.geometry(P8.mesh.coords, P8.mesh.tets, P8.mesh.bfaces)
    kt = np.log(P8.kappa / P8.kappa0)
    mt = np.log(P8.mu / P8.mu0)
    delta = 1e-6
    Pd = prior.Prior(g, kt, mt, T, 1.0, delta, solver="deflated")
    Pl = prior.Prior(g, kt, mt, T, 1.0, delta, solver="direct")
    p = np.random.default_rng(6).standard_normal(2 * g.N)
    xd, xl = Pd.solve(p), Pl.solve(p)
    res_d = np.linalg.norm(_ideal_residual(Pd.Md, g.N, xd, p, delta)) / np.linalg.norm(p)
    assert res_d <= 1e-10
    N = g.N
    for j in range(2):
        mj = p[j * N:(j + 1) * N].mean() / delta
        assert abs(xd[j * N:(j + 1) * N].mean() - mj) <= 1e-13 * abs(mj)
    assert np.linalg.norm(xd - xl) / np.linalg.norm(xd) <= 1e-7
