"""Pins of the oracle's Voronoi (Eq. 3-5) and circumcentre (Eq. 6) scalar
operators (CPU only). The oracle builds them from the geometry the
equations name (circumcentres, edge midpoints, the quasi-hexagonal cells);
the pins use angles, closed forms and continuum limits instead."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W


def _angles_cot(mesh):
    act = O.active_cells(mesh)
    tris = np.asarray(mesh.tris)[act]
    a, b, c = O.operators._corner_positions(mesh, tris)
    P = (a, b, c)
    cot = []
    for k in range(3):
        u, v = P[(k + 1) % 3] - P[k], P[(k + 2) % 3] - P[k]
        cot.append(np.sum(u * v, 1) / O.operators._cross_norm(u, v))
    return tris, P, cot


@pytest.mark.parametrize("mesh", ["planar", "sphere"])
def test_voronoi_flux_weights_are_cotangent_weights(mesh):
    """Eq. 3's l/d across an edge is (cot a + cot b) / 2, the P1 weight
    (Sect. 2.1.1), so the Voronoi and the FE stiffness agree."""
    m = W.split_square(12, jitter=0.12) if mesh == "planar" else W.icosphere(3, jitter=0.1)
    vo = O.voronoi_operator(m, 1)
    K, *_ = O.cot_stiffness(m)
    assert abs(vo.K - K).max() <= 1e-13 * abs(K).max()


def test_voronoi_cell_areas_from_angles():
    """The circumcentric cell of corner i of triangle (i, j, k) has area
    (|ij|^2 cot(theta_k) + |ik|^2 cot(theta_j)) / 8; the cells tile the
    mesh."""
    m = W.split_square(10, jitter=0.15)
    vo = O.voronoi_operator(m, 1)
    tris, P, cot = _angles_cot(m)
    A = np.zeros(m.n_vertices)
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        lij = np.sum((P[j] - P[i]) ** 2, 1)
        lik = np.sum((P[k] - P[i]) ** 2, 1)
        np.add.at(A, tris[:, i], (lij * cot[k] + lik * cot[j]) / 8.0)
    assert np.allclose(vo.A, A[vo.verts], rtol=1e-12, atol=0)
    assert abs(vo.A.sum() / 100.0 - 1) < 1e-13


@pytest.mark.parametrize("n_order", [1, 2])
def test_voronoi_equals_fe_on_uniform_mesh(n_order):
    """Sect. 2.1.1 below Eq. 4: on uniform meshes (M^L)^-1 D~ = D, i.e. the
    Voronoi cells are the median-dual ones and the operators coincide."""
    m = W.split_square(16, jitter=0.0)
    vo, so = O.voronoi_operator(m, n_order), O.scalar_operator(m, n_order)
    assert np.allclose(vo.A, so.A, rtol=1e-14, atol=0)
    assert abs(vo.Kn - so.Kn).max() <= 1e-13


def _equilateral_periodic(n, rows):
    h = math.sqrt(3) / 2
    coords = np.array([[i + 0.5 * (j % 2), j * h] for j in range(rows) for i in range(n)])

    def v(i, j):
        return (i % n) + n * (j % rows)

    tris = []
    for j in range(rows):
        for i in range(n):
            if j % 2 == 0:
                tris += [(v(i, j), v(i + 1, j), v(i, j + 1)), (v(i + 1, j), v(i + 1, j + 1), v(i, j + 1))]
            else:
                tris += [(v(i, j), v(i + 1, j), v(i + 1, j + 1)), (v(i, j), v(i + 1, j + 1), v(i, j + 1))]
    return W.Mesh(coords=coords, tris=np.array(tris, dtype=np.int32), geometry=W.GEOM_PERIODIC,
                  period=(float(n), rows * h), h=1.0)


def test_circumcenter_equilateral_weights_and_continuum_limit():
    """Eq. 6 on equilateral triangles of unit edge: neighbouring
    circumcentres are 1/sqrt(3) apart, so every weight is sqrt(3) and the
    cell area sqrt(3)/4; the Bloch symbol of A^-1 K over the two triangle
    orientations tends to |q|^2 (the operator is -Laplacian)."""
    m = _equilateral_periodic(6, 6)
    co = O.circumcenter_operator(m, 1)
    off = (co.K - sp.diags(co.K.diagonal())).tocsr()
    off.eliminate_zeros()
    assert np.allclose(off.data, -math.sqrt(3), rtol=1e-13)
    assert np.allclose(co.A, math.sqrt(3) / 4, rtol=1e-13)
    x = m.coords
    t = m.tris
    cen = np.zeros((t.shape[0], 2))
    for k in range(3):  # centroid = circumcentre on equilateral triangles
        d = x[t[:, k]] - x[t[:, 0]]
        d -= np.asarray(m.period) * np.round(d / np.asarray(m.period))
        cen += (x[t[:, 0]] + d) / 3.0
    K = co.K.tocsr()
    for th in np.linspace(0, np.pi, 5):
        q = 0.01 * np.array([math.cos(th), math.sin(th)])
        H = np.zeros((2, 2), dtype=complex)
        for a, ca in enumerate((0, 1)):
            row = K.getrow(ca)
            for cb, val in zip(row.indices, row.data):
                d = cen[cb] - cen[ca]
                d -= np.asarray(m.period) * np.round(d / np.asarray(m.period))
                H[a, cb % 2] += val * np.exp(1j * (q @ d))
        lam = np.linalg.eigvalsh(H / co.A[0]).min()
        assert abs(lam / (q @ q) - 1) < 1e-3


def test_circumcenter_operator_invariants():
    """Symmetric, zero row sums, positive semi-definite (a weighted graph
    Laplacian with positive weights on a well-centred mesh)."""
    s = W.icosphere(3, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    co = O.circumcenter_operator(s, 2)
    K = co.K
    assert abs(K - K.T).max() == 0
    assert abs(np.asarray(K.sum(1))).max() <= 1e-13 * abs(K).max()
    off = (K - sp.diags(K.diagonal())).tocsr()
    assert np.all(off.data <= 0)
    ev = np.linalg.eigvalsh(K.toarray())
    assert ev.min() >= -1e-12 * ev.max()
    assert np.allclose(co.A.sum(), O.scalar_operator(s, 1).A.sum(), rtol=1e-13)
