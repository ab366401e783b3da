"""Pins of the oracle's vertex FE vector Laplacian (Sect. 2.1.2):
D_2 = [[D~, T], [-T, D~]] with metric factor m = tan(latitude) / R_e.

The operator's continuum limit is fixed by differential geometry: its
quadratic form is sum (d_x u - m v)^2 + (d_x v + m u)^2 + |d_y u|^2 +
|d_y v|^2 + R_e^-2 |u|^2, the covariant (rough) energy plus the curvature
term, i.e. the Hodge Laplacian on tangent fields of the sphere, whose
eigenvalues are l (l + 1) / R_e^2 (l >= 1) for both rotational and
gradient fields. Lon/lat components are singular at the poles, so the
eigen-pins use fields that are smooth in components (rotation about the
polar axis) or test fields windowed away from the poles (weak residual).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W


def _frames(op, s):
    P = s.coords[op.verts]
    ph = P / np.linalg.norm(P, axis=1, keepdims=True)
    cl = np.hypot(ph[:, 0], ph[:, 1])
    ee = np.stack([-ph[:, 1], ph[:, 0], np.zeros_like(cl)], axis=1) / cl[:, None]
    en = np.cross(ph, ee)
    return ph, cl, ee, en


def _components(X, ee, en):
    return np.stack([np.sum(X * ee, axis=1), np.sum(X * en, axis=1)], axis=1).ravel()


def test_planar_mesh_gives_two_decoupled_scalar_laplacians():
    """On planar meshes m = 0 and 1/R_e^2 = 0: D~ is the scalar stiffness and
    T = 0, so each component is the scalar filter of Sect. 2.1.1."""
    m = W.split_square(16, jitter=0.2)
    sc = O.scalar_operator(m, 2)
    vv = O.vertex_vector_operator(m, 2)
    for comp in range(2):
        blk = vv.Kn[comp::2, :][:, comp::2]
        assert abs(blk - sc.Kn).max() <= 1e-14 * abs(sc.Kn).max()
        assert vv.Kn[comp::2, :][:, 1 - comp::2].nnz == 0 or abs(vv.Kn[comp::2, :][:, 1 - comp::2]).max() == 0
    assert np.array_equal(vv.A[0::2], sc.A) and np.array_equal(vv.A[1::2], sc.A)


def test_symmetric_positive_definite_masked_sphere():
    """T is antisymmetric, so D_2 is symmetric; the curvature term makes it
    positive definite (smallest eigenvalue ~ 2/R_e^2 times the mass)."""
    s = W.icosphere(3, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    op = O.vertex_vector_operator(s, 1)
    D = op.K
    assert abs(D - D.T).max() <= 1e-15 * abs(D).max()
    T = D[0::2, :][:, 1::2]
    assert abs(T + T.T).max() <= 1e-15 * abs(D).max()
    assert abs(T.diagonal()).max() == 0.0
    Dm = (sp.diags(1 / np.sqrt(op.A)) @ D @ sp.diags(1 / np.sqrt(op.A))).toarray()
    ev = np.linalg.eigvalsh(Dm)
    assert ev.min() > 0.5 / s.radius ** 2


def test_solid_body_rotation_is_an_eigenfield():
    """Rotation about the polar axis (u = cos(latitude), v = 0, smooth in
    components): the Rayleigh quotient tends to 2/R_e^2 at second order
    (checks the gradient, m^2 and R_e^-2 terms)."""
    errs = []
    for level in (4, 5):
        s = W.icosphere(level, jitter=0.1)
        op = O.vertex_vector_operator(s, 1)
        ph, cl, ee, en = _frames(op, s)
        x = _components(np.cross([0.0, 0.0, 1.0], ph), ee, en)
        q = (x @ (op.K @ x)) / (x @ (op.A * x)) * s.radius ** 2
        errs.append(abs(q - 2.0))
    assert errs[0] < 6e-3
    assert errs[1] < errs[0] / 3.0


def _hodge_fields(ph):
    w = np.array([0.3, -0.5, 0.8])
    w /= np.linalg.norm(w)
    a = np.array([1.0, 0.2, 0.1])
    a /= np.linalg.norm(a)
    b = np.cross(a, [0.1, 0.7, 0.3])
    b /= np.linalg.norm(b)

    def tang(v):
        return v - np.sum(v * ph, axis=1, keepdims=True) * ph

    # gradient of the l = 2 harmonic (p.a)(p.b), a _|_ b
    g2 = np.sum(ph * b, axis=1)[:, None] * tang(np.broadcast_to(a, ph.shape)) + \
        np.sum(ph * a, axis=1)[:, None] * tang(np.broadcast_to(b, ph.shape))
    return {"rotation l=1": (np.cross(w, ph), 2.0), "gradient l=1": (tang(np.broadcast_to(w, ph.shape)), 2.0),
            "gradient l=2": (g2, 6.0), "rotation l=2": (np.cross(ph, g2), 6.0)}


@pytest.mark.parametrize("field", ["rotation l=1", "gradient l=1", "gradient l=2", "rotation l=2"])
def test_tilted_hodge_eigenfields_weak_residual(field):
    """Tilted l = 1 and l = 2 eigenfields (rotational and gradient, both
    components non-zero, so T is exercised) against a test field windowed
    by cos^4(latitude): y^T (D_2 x - lambda M_2 x) / (lambda y^T M_2 x) is a
    Galerkin residual, second order in h. A wrong sign of T, a missing T,
    m^2 or R_e^-2 term each give 1e-2 or more."""
    res = []
    for level in (4, 5):
        s = W.icosphere(level, jitter=0.1)
        op = O.vertex_vector_operator(s, 1)
        ph, cl, ee, en = _frames(op, s)
        X, l = _hodge_fields(ph)[field]
        x = _components(X, ee, en)
        lam = l / s.radius ** 2
        y = np.repeat(cl ** 4, 2) * x
        res.append(abs((y @ (op.K @ x) - lam * (y @ (op.A * x))) / (lam * (y @ (op.A * x)))))
    assert res[0] < (3e-4 if field.endswith("l=1") else 3e-3)
    assert res[1] < res[0] / 3.0


def test_single_triangle_by_quadrature():
    """One spherical triangle, entries recomputed by the edge-midpoint rule
    (exact for the quadratic integrands): N_i from barycentric coordinates,
    the facet gradient by least squares on the two edge vectors, d_x along
    the zonal direction at the centroid, m = tan(latitude) / R_e."""
    R = 6371.0
    lat = np.radians([40.0, 41.5, 40.7])
    lon = np.radians([10.0, 10.4, 11.3])
    P = R * np.stack([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)], axis=1)
    mesh = W.Mesh(coords=np.ascontiguousarray(P), tris=np.array([[0, 1, 2]], dtype=np.int32),
                  geometry=O.operators.GEOM_SPHERE, h=1.0, radius=R, name="one")
    op = O.vertex_vector_operator(mesh, 1)
    E = np.stack([P[1] - P[0], P[2] - P[0]], axis=1)  # 3 x 2
    area = 0.5 * np.linalg.norm(np.cross(E[:, 0], E[:, 1]))
    dN = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])  # N_i(b) - N_i(a), N_i(c) - N_i(a)
    grads = [E @ np.linalg.solve(E.T @ E, dN[i]) for i in range(3)]
    cen = P.mean(axis=0)
    clat = np.arcsin(cen[2] / np.linalg.norm(cen))
    clon = np.arctan2(cen[1], cen[0])
    east = np.array([-np.sin(clon), np.cos(clon), 0.0])
    m = np.tan(clat) / R
    dx = [g @ east for g in grads]
    mids = [(0, 1), (1, 2), (2, 0)]
    Nmid = np.array([[0.5 if i in e else 0.0 for e in mids] for i in range(3)])  # N_i at the midpoints

    def quad(f):  # f: values at the three edge midpoints
        return area / 3.0 * np.sum(f)

    D = np.zeros((6, 6))
    for i in range(3):
        for j in range(3):
            dt = area * grads[i] @ grads[j] + (1 / R ** 2 + m ** 2) * quad(Nmid[i] * Nmid[j])
            t = quad(m * (-Nmid[j] * dx[i] + Nmid[i] * dx[j]))
            D[2 * i, 2 * j] = D[2 * i + 1, 2 * j + 1] = dt
            D[2 * i, 2 * j + 1] = t
            D[2 * i + 1, 2 * j] = -t
    got = op.K.toarray()
    assert np.max(np.abs(got - D)) <= 1e-12 * np.max(np.abs(D))
    assert np.allclose(op.A, area / 3.0, rtol=1e-14)
    assert np.allclose(op.Rvc.toarray(), np.kron(np.ones((3, 1)), np.eye(2)) * area / 3.0, rtol=1e-14)


def test_projection_and_filter_limits():
    """R_vc distributes A_c u_c to the corners (totals conserved); a
    constant cell field on a planar mesh projects to the constant; as
    k -> infinity the filter returns M_2^-1 R_vc u_c and the filter is
    linear."""
    m = W.split_square(12, jitter=0.2)
    op = O.vertex_vector_operator(m, 1)
    u = np.tile([0.7, -1.3], (m.n_triangles, 1))
    b = O.project_cells_to_vertices(op, u)
    assert np.allclose(b / op.A, np.tile([0.7, -1.3], op.verts.size), rtol=1e-14)
    s = W.icosphere(3, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    op = O.vertex_vector_operator(s, 1)
    u = W.sphere_k3_velocity(s, 3, 4, n_waves=64)
    b = O.project_cells_to_vertices(op, u)
    act = O.active_cells(s)
    area = op.Rvc.sum(axis=0).A1.reshape(-1, 2)[:, 0]
    assert np.allclose(b.reshape(-1, 2).sum(axis=0), (area[:, None] * u).sum(axis=0), rtol=1e-12)
    assert np.all(area[~act] == 0)
    out = O.filter_vertex_vector(op, u, [1e9 / s.h])
    assert np.allclose(out[0][op.verts].ravel(), b / op.A, rtol=1e-12, atol=1e-15)
    u2 = W.sphere_k3_velocity(s, 5, 6, n_waves=64)
    ks = W.log_scales(s.h, 2)
    o1, o2, o3 = (O.filter_vertex_vector(op, f, ks) for f in (u, u2, 2 * u - u2))
    assert np.max(np.abs(o3 - (2 * o1 - o2))) <= 1e-12 * np.max(np.abs(o1))
