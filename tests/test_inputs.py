"""Input generator: Kuhn mesh topology, phantoms and sources."""
import itertools

import numpy as np
import pytest

from qpat_inputs import kuhn_mesh, make_problem, gaussian_sources, face_sources
from qpat_inputs.sources import gaussian_centre


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_kuhn_counts(n):
    m = kuhn_mesh(n, 40.0)
    assert m.N == (n + 1) ** 3
    assert m.E == 6 * n ** 3
    assert m.F_b == 12 * n ** 2
    # every tetrahedron has volume h^3/6
    x = m.coords[m.tets]
    vol = np.abs(np.linalg.det(x[:, 1:] - x[:, :1])) / 6.0
    assert np.allclose(vol, m.h ** 3 / 6.0, rtol=1e-12)


@pytest.mark.parametrize("n", [2, 3])
def test_kuhn_conforming_and_boundary(n):
    """Interior faces are shared by exactly two tetrahedra; the listed boundary
    triangles are exactly the faces used once (brute force)."""
    m = kuhn_mesh(n, 40.0)
    count = {}
    for t in m.tets:
        for f in itertools.combinations(sorted(t.tolist()), 3):
            count[f] = count.get(f, 0) + 1
    assert max(count.values()) == 2
    once = {f for f, c in count.items() if c == 1}
    listed = {tuple(sorted(f.tolist())) for f in m.bfaces}
    assert once == listed
    assert len(listed) == m.F_b


@pytest.mark.parametrize("n", [2, 4])
def test_kuhn_edges_and_nnz(n):
    """14 neighbours per interior node; nnz = N + 2 (3n(n+1)^2 + 3n^2(n+1) + n^3)."""
    m = kuhn_mesh(n, 40.0)
    edges = set()
    for t in m.tets:
        for a, b in itertools.combinations(t.tolist(), 2):
            edges.add((min(a, b), max(a, b)))
    nnz = m.N + 2 * len(edges)
    assert nnz == m.N + 2 * (3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3)
    deg = np.zeros(m.N, int)
    for a, b in edges:
        deg[a] += 1
        deg[b] += 1
    assert deg.max() == 14


def test_face_sources_indicator():
    m = kuhn_mesh(3, 40.0)
    src = face_sources(m, [0, 3])
    assert src.shape == (2, m.F_b, 3)
    assert np.all(src[0][m.bface_tag == 0] == 1.0)
    assert np.all(src[0][m.bface_tag != 0] == 0.0)
    assert np.all(src[1][m.bface_tag == 3] == 1.0)


def test_gaussian_sources_centres():
    m = kuhn_mesh(8, 40.0)
    face, c = gaussian_centre(m, 0)
    assert face == 0 and np.allclose(c, [20, 20, 0])
    face, c = gaussian_centre(m, 3)
    assert face == 3 and np.allclose(c, [40, 20, 20])
    face, c = gaussian_centre(m, 6)
    assert face == 0 and np.allclose(c, [30, 20, 0])
    src = gaussian_sources(m, 8)
    # peak value 1 at the vertex closest to the centre of face -z
    assert np.isclose(src[0].max(), 1.0)
    assert np.all(src[0][m.bface_tag != 0] == 0.0)


def test_problem_seeded_and_physical():
    a = make_problem("T8")
    b = make_problem("T8")
    assert np.array_equal(a.kappa, b.kappa) and np.array_equal(a.mu, b.mu)
    assert np.all(a.mu > 0) and np.all(a.kappa > 0)
    assert np.allclose(a.kappa, 1.0 / (3.0 * (a.mua + a.mus)))
    c1 = make_problem("C1")
    assert c1.mesh.N == 4913 and c1.n_ill == 4
    assert set(np.unique(c1.mu)) <= {0.01, 0.02}


def test_coarse_in_fine_maps_nodes_onto_nodes():
    from qpat_inputs import coarse_in_fine
    for n in (1, 3, 8):
        c, f = kuhn_mesh(n, 40.0), kuhn_mesh(2 * n, 40.0)
        idx = coarse_in_fine(n)
        assert idx.shape == (c.N,) and len(np.unique(idx)) == c.N
        assert np.array_equal(f.coords[idx], c.coords)


def test_illumination_study_phantom_fits_the_small_cube():
    """S2: the same shapes at n and 2n (same seed), inside the 11 mm cube."""
    from qpat_inputs import coarse_in_fine
    P, Pf = make_problem("S2", n=8), make_problem("S2", n=16)
    assert P.mesh.coords.max() == 11.0 and P.n_ill == 3
    assert np.array_equal(Pf.mu[coarse_in_fine(8)], P.mu)
    assert P.mu.max() > P.mu0 * 1.2        # an inclusion is resolved
