"""Discrete operators of the implicit filter (oracle, FP64, test-only).

Scalar placement on vertices (median-dual control volumes, P1 elements),
Sect. 2.1.1 "Scalar Laplacians":

* Galerkin weak form ``(M + (1/2) D~) phi_bar = M phi`` with
  ``D~_vv' = l^2 int grad N_v . grad N_v'``; here ``K = D~ / l^2`` is the
  l-free P1 stiffness, so ``S(k) = M + gamma k^-2 K`` with ``k = 1/l``.
* ``M`` is replaced by its lumped form ``A_v I`` (median-dual area).
* Biharmonic: ``S = M + (1/2) D~ (M^L)^-1 D~``; in general the order-n
  operator is ``K_n = K (M^-1 K)^(n-1)``.
* The finite-volume treatment (triangle gradients, fluxes through the
  median-dual segments) gives the same matrix; ``fv_stiffness`` builds it
  that way, independently, for the tests.

Cell placement for vectors, Sect. 2.1.2 "Vector Laplacians", Eq. 7:
``A_c (D u)_c = A l^2 sum_{c' in C(c)} (u_c - u_c')`` over edge neighbours,
with the change of the local (east, north) unit vectors between ``c`` and
``c'`` accounted for on the sphere.

Boundary conditions of no normal flux (Sect. 2.1, below Eq. 2) are the
natural conditions of the weak form: only active triangles are assembled.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

GEOM_PLANAR = 0
GEOM_PERIODIC = 1
GEOM_SPHERE = 2


def active_cells(mesh) -> np.ndarray:
    """A triangle takes part iff its three vertices are wet (land-mask
    convention); returns a bool mask over triangles."""
    if mesh.wet is None:
        return np.ones(mesh.tris.shape[0], dtype=bool)
    w = np.asarray(mesh.wet).astype(bool)
    t = mesh.tris
    return w[t[:, 0]] & w[t[:, 1]] & w[t[:, 2]]


def _corner_positions(mesh, tris):
    """Positions of the three corners of each triangle, with periodic
    edges unwrapped by the minimum image relative to corner 0."""
    x = np.asarray(mesh.coords, dtype=np.float64)
    a = x[tris[:, 0]]
    b = x[tris[:, 1]]
    c = x[tris[:, 2]]
    if mesh.geometry == GEOM_PERIODIC:
        p = np.asarray(mesh.period, dtype=np.float64)
        b = a + ((b - a) - p * np.round((b - a) / p))
        c = a + ((c - a) - p * np.round((c - a) / p))
    return a, b, c


def _cross_norm(u, v):
    if u.shape[1] == 2:
        return np.abs(u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0])
    return np.linalg.norm(np.cross(u, v), axis=1)


def _dof_numbering(n_vertices, tris):
    """Dofs = vertices of at least one active triangle, numbered in
    increasing vertex id."""
    used = np.zeros(n_vertices, dtype=bool)
    used[tris.ravel()] = True
    verts = np.nonzero(used)[0]
    dof_of = np.full(n_vertices, -1, dtype=np.int64)
    dof_of[verts] = np.arange(verts.size)
    return verts, dof_of


def cot_stiffness(mesh):
    """P1 stiffness ``K_vv' = int grad N_v . grad N_v'`` by the cotangent
    formula (Sect. 2.1.1): a triangle with corners i, j, l adds
    ``-cot(theta_l)/2`` to ``K_ij`` and ``K_ji`` (``theta_l`` the angle
    opposite edge ij) and ``(cot theta_j + cot theta_l)/2`` to ``K_ii``.
    Triangle areas are those of the flat facets.

    Returns ``(K, areas, verts, dof_of, tris_active)`` with ``K`` a CSR
    matrix over dofs and ``areas`` the flat-facet triangle areas.
    """
    act = active_cells(mesh)
    tris = np.asarray(mesh.tris, dtype=np.int64)[act]
    verts, dof_of = _dof_numbering(mesh.n_vertices, tris)
    a, b, c = _corner_positions(mesh, tris)
    P = (a, b, c)
    idx = dof_of[tris]
    rows, cols, vals = [], [], []
    area = 0.5 * _cross_norm(b - a, c - a)
    cot = []
    for l in range(3):
        i, j = (l + 1) % 3, (l + 2) % 3
        u = P[i] - P[l]
        v = P[j] - P[l]
        cot.append(np.sum(u * v, axis=1) / _cross_norm(u, v))
    for l in range(3):
        i, j = (l + 1) % 3, (l + 2) % 3
        w = -0.5 * cot[l]
        rows += [idx[:, i], idx[:, j]]
        cols += [idx[:, j], idx[:, i]]
        vals += [w, w]
    for i in range(3):
        j, l = (i + 1) % 3, (i + 2) % 3
        rows.append(idx[:, i])
        cols.append(idx[:, i])
        vals.append(0.5 * (cot[j] + cot[l]))
    n = verts.size
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    K.sort_indices()
    return K, area, verts, dof_of, tris


def fv_stiffness(mesh):
    """Finite-volume route to the same matrix (Sect. 2.1.1, last paragraph
    on scalar Laplacians): the gradient of the linear interpolant is found
    on each triangle from its three vertex values, and ``-grad phi . n`` is
    integrated over the two median-dual segments inside the triangle
    (edge midpoint -> centroid -> other edge midpoint) around each corner.
    On the sphere each flat facet is handled in its own 2-D frame.
    Returns the CSR matrix over the same dof numbering as ``cot_stiffness``.
    """
    act = active_cells(mesh)
    tris = np.asarray(mesh.tris, dtype=np.int64)[act]
    verts, dof_of = _dof_numbering(mesh.n_vertices, tris)
    a, b, c = _corner_positions(mesh, tris)
    if a.shape[1] == 3:
        t1 = b - a
        t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
        nrm = np.cross(b - a, c - a)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        t2 = np.cross(nrm, t1)

        def loc(p):
            d = p - a
            return np.stack([np.sum(d * t1, axis=1), np.sum(d * t2, axis=1)], axis=1)

        a2, b2, c2 = loc(a), loc(b), loc(c)
    else:
        a2, b2, c2 = a, b, c
    P = [a2, b2, c2]
    # gradient operator G (F, 2, 3): [x1-x0; x2-x0] g = [phi1-phi0; phi2-phi0]
    E = np.stack([b2 - a2, c2 - a2], axis=1)  # (F, 2, 2) rows are edge vectors
    Einv = np.linalg.inv(E)
    Dm = np.array([[-1.0, 1.0, 0.0], [-1.0, 0.0, 1.0]])
    G = Einv @ Dm  # (F, 2, 3)
    cen = (a2 + b2 + c2) / 3.0
    idx = dof_of[tris]
    rows, cols, vals = [], [], []

    def outward(p, q):
        d = q - p
        return np.stack([d[:, 1], -d[:, 0]], axis=1)  # right normal of p->q

    for i in range(3):
        j, l = (i + 1) % 3, (i + 2) % 3
        m_ij = 0.5 * (P[i] + P[j])
        m_il = 0.5 * (P[i] + P[l])
        # corner i's part of its control volume is i -> m_ij -> cen -> m_il (CCW)
        s = outward(m_ij, cen) + outward(cen, m_il)
        flux = -np.einsum("fd,fdk->fk", s, G)  # (F, 3) coefficients of phi_T
        for kk in range(3):
            rows.append(idx[:, i])
            cols.append(idx[:, kk])
            vals.append(flux[:, kk])
    n = verts.size
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    K.sort_indices()
    return K


def lumped_mass(n_dofs, dof_tris, areas):
    """Lumped mass ``M^L = A_v I``: ``A_v`` is the median-dual control
    volume area, one third of the area of every active triangle touching
    ``v`` (Sect. 2.1.1)."""
    A = np.zeros(n_dofs, dtype=np.float64)
    for k in range(3):
        np.add.at(A, dof_tris[:, k], areas / 3.0)
    return A


def order_n(K, A, n: int):
    """Order-n operator ``K_n = K (M^-1 K)^(n-1)`` (n = 1: the Laplacian
    form; n = 2: the biharmonic ``D~ (M^L)^-1 D~`` form, Sect. 2.1.1 and
    Eq. 5, with flux terms omitted by the boundary conditions)."""
    Kn = K.tocsr()
    Minv = sp.diags(1.0 / A)
    for _ in range(n - 1):
        Kn = (Kn @ (Minv @ K)).tocsr()
    Kn.sort_indices()
    return Kn


@dataclasses.dataclass
class ScalarOperator:
    """Vertex-scalar operator: ``K_n`` over dofs, lumped mass ``A``, and
    the vertex <-> dof maps (``verts[d]`` is dof d's vertex)."""

    K: sp.csr_matrix
    Kn: sp.csr_matrix
    A: np.ndarray
    n: int
    verts: np.ndarray
    dof_of: np.ndarray
    n_vertices: int


def scalar_operator(mesh, n: int = 1) -> ScalarOperator:
    K, area, verts, dof_of, tris = cot_stiffness(mesh)
    A = lumped_mass(verts.size, dof_of[tris], area)
    Kn = order_n(K, A, n)
    return ScalarOperator(K=K, Kn=Kn, A=A, n=n, verts=verts, dof_of=dof_of, n_vertices=mesh.n_vertices)


@dataclasses.dataclass
class VectorOperator:
    """Cell-vector operator of Eq. 7 over active triangles, unknowns
    interleaved ``(u_c, v_c)`` as ``2c, 2c+1``; ``A`` holds the cell areas
    repeated per component."""

    K: sp.csr_matrix
    Kn: sp.csr_matrix
    A: np.ndarray
    n: int
    cells: np.ndarray
    n_cells_total: int


def _cell_frames(mesh, a, b, c):
    """(east, north) unit vectors at each cell: on the sphere
    ``e_E = z x c / |z x c|`` and ``e_N = c x e_E`` at the centroid
    direction ``c``; on planar meshes the x and y axes."""
    nf = a.shape[0]
    if mesh.geometry != GEOM_SPHERE:
        ee = np.tile(np.array([1.0, 0.0, 0.0]), (nf, 1))
        en = np.tile(np.array([0.0, 1.0, 0.0]), (nf, 1))
        return ee, en
    cd = a + b + c
    cd /= np.linalg.norm(cd, axis=1, keepdims=True)
    z = np.array([0.0, 0.0, 1.0])
    ee = np.cross(np.broadcast_to(z, cd.shape), cd)
    ee /= np.linalg.norm(ee, axis=1, keepdims=True)
    en = np.cross(cd, ee)
    return ee, en


def vector_operator(mesh, n: int = 1, stencil_A: float = np.sqrt(3.0)) -> VectorOperator:
    """Eq. 7 on active triangles with edge neighbours ``C(c)``:
    ``(K u)_c = A sum_{c'} (u_c - P_cc' u_c')`` where
    ``P_cc' = [[eE_c.eE_c', eE_c.eN_c'], [eN_c.eE_c', eN_c.eN_c']]`` maps the
    components at ``c'`` into the frame at ``c`` (the metric terms from the
    change of unit vectors; on planar meshes ``P = I``). Mass: cell areas.

    Parity unpinned for the exact metric-term formula on the sphere (the
    paper gives no formula); pinned by symmetry, PSD, the planar limit and
    the printed continuum limits of the stencil constant ``A``.
    """
    act = active_cells(mesh)
    cells = np.nonzero(act)[0]
    tris = np.asarray(mesh.tris, dtype=np.int64)[act]
    a, b, c = _corner_positions(mesh, tris)
    area = 0.5 * _cross_norm(b - a, c - a)
    ee, en = _cell_frames(mesh, a, b, c)
    nc = tris.shape[0]
    # edge -> the (one or two) active cells that own it
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], axis=0)
    owner = np.concatenate([np.arange(nc)] * 3)
    key = np.minimum(e[:, 0], e[:, 1]) * mesh.n_vertices + np.maximum(e[:, 0], e[:, 1])
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = ks[1:] == ks[:-1]
    c1 = owner[order][:-1][same]
    c2 = owner[order][1:][same]
    rows, cols, vals = [], [], []
    deg = np.zeros(nc)
    np.add.at(deg, c1, 1.0)
    np.add.at(deg, c2, 1.0)
    for comp in range(2):
        rows.append(2 * np.arange(nc) + comp)
        cols.append(2 * np.arange(nc) + comp)
        vals.append(stencil_A * deg)
    Fr = [ee, en]
    for (p, q) in ((c1, c2), (c2, c1)):
        for r in range(2):
            for s in range(2):
                rows.append(2 * p + r)
                cols.append(2 * q + s)
                vals.append(-stencil_A * np.sum(Fr[r][p] * Fr[s][q], axis=1))
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * nc, 2 * nc)).tocsr()
    K.sort_indices()
    A2 = np.repeat(area, 2)
    Kn = order_n(K, A2, n)
    return VectorOperator(K=K, Kn=Kn, A=A2, n=n, cells=cells, n_cells_total=mesh.n_triangles)


# ------------------------------------------------------------ Eq. 3-6
def _circumcentric_geometry(a, b, c):
    """Per triangle (corners a, b, c, flat facet, 2-D or 3-D): the corners
    and circumcentre in 3-D, the unit normal of (b - a) x (c - a) and, for
    each edge k (opposite corner k), the signed distance from the edge's
    midpoint to the circumcentre, measured in the facet's plane towards
    corner k, the edge length and the midpoint. Computed from the
    circumcentre's coordinates (not from angles)."""
    if a.shape[1] == 2:
        z = np.zeros((a.shape[0], 1))
        a, b, c = np.hstack([a, z]), np.hstack([b, z]), np.hstack([c, z])
    ab, ac = b - a, c - a
    nrm = np.cross(ab, ac)
    n2 = np.sum(nrm * nrm, axis=1, keepdims=True)
    O = a + (np.sum(ac * ac, 1, keepdims=True) * np.cross(nrm, ab) +
             np.sum(ab * ab, 1, keepdims=True) * np.cross(ac, nrm)) / (2.0 * n2)
    P = (a, b, c)
    unit_n = nrm / np.sqrt(n2)
    dist, length, mids = [], [], []
    for k in range(3):
        i, j = (k + 1) % 3, (k + 2) % 3
        e = P[j] - P[i]
        le = np.linalg.norm(e, axis=1)
        mid = 0.5 * (P[i] + P[j])
        u = np.cross(unit_n, e) / le[:, None]  # in-plane, perpendicular to the edge
        u *= np.sign(np.sum(u * (P[k] - mid), axis=1))[:, None]  # towards corner k
        dist.append(np.sum((O - mid) * u, axis=1))
        length.append(le)
        mids.append(mid)
    return O, P, unit_n, dist, length, mids


def voronoi_operator(mesh, n: int = 1) -> ScalarOperator:
    """Scalars on vertices with quasi-hexagonal (Voronoi) control volumes,
    Eq. 3-5: ``A_v (D phi)_v = l^2 sum_v' (phi_v - phi_v') l_vv' / d_vv'``
    with ``d`` the edge length and ``l`` the distance between the
    circumcentres on both sides of the edge (through the edge midpoint;
    only the side of an active triangle counts, so boundary edges take one
    segment), and ``A_v`` the area of the circumcentric cell: over the
    active triangles at v, the quadrilaterals (v, midpoint, circumcentre,
    midpoint)."""
    act = active_cells(mesh)
    tris = np.asarray(mesh.tris, dtype=np.int64)[act]
    verts, dof_of = _dof_numbering(mesh.n_vertices, tris)
    a, b, c = _corner_positions(mesh, tris)
    O, P, unit_n, dist, length, mids = _circumcentric_geometry(a, b, c)
    idx = dof_of[tris]
    nv = verts.size
    rows, cols, vals = [], [], []
    diag = np.zeros(nv)
    for k in range(3):
        i, j = (k + 1) % 3, (k + 2) % 3
        w = dist[k] / length[k]
        rows += [idx[:, i], idx[:, j]]
        cols += [idx[:, j], idx[:, i]]
        vals += [-w, -w]
        np.add.at(diag, idx[:, i], w)
        np.add.at(diag, idx[:, j], w)
    rows.append(np.arange(nv))
    cols.append(np.arange(nv))
    vals.append(diag)
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nv, nv)).tocsr()
    K.sort_indices()
    A = np.zeros(nv)
    for i in range(3):
        # corners (i, j, k) run the same way round as (a, b, c), and so does
        # the quadrilateral (corner, midpoint of ij, circumcentre, midpoint
        # of ik): its area is positive unless the circumcentre lies outside
        j, k = (i + 1) % 3, (i + 2) % 3
        m_ij, m_ik, pi = mids[k], mids[j], P[i]
        quad = 0.5 * (np.sum(np.cross(m_ij - pi, O - pi) * unit_n, 1) + np.sum(np.cross(O - pi, m_ik - pi) * unit_n, 1))
        np.add.at(A, idx[:, i], quad)
    Kn = order_n(K, A, n)
    return ScalarOperator(K=K, Kn=Kn, A=A, n=n, verts=verts, dof_of=dof_of, n_vertices=mesh.n_vertices)


@dataclasses.dataclass
class CellScalarOperator:
    """Scalars at triangle circumcentres (Eq. 6) over active triangles."""

    K: sp.csr_matrix
    Kn: sp.csr_matrix
    A: np.ndarray
    n: int
    cells: np.ndarray
    n_cells_total: int


def circumcenter_operator(mesh, n: int = 1) -> CellScalarOperator:
    """Eq. 6: ``A_c (D phi)_c = l^2 sum_c' (phi_c - phi_c') l_cc' / d_cc'`` over
    the active triangles c' sharing an edge with c, ``l_cc'`` the length of
    that edge and ``d_cc'`` the distance between the two circumcentres
    (through the edge midpoint); ``A_c`` the triangle's area."""
    act = active_cells(mesh)
    cells = np.nonzero(act)[0]
    tris = np.asarray(mesh.tris, dtype=np.int64)[act]
    a, b, c = _corner_positions(mesh, tris)
    area = 0.5 * _cross_norm(b - a, c - a)
    O, P, unit_n, dist, length, mids = _circumcentric_geometry(a, b, c)
    nc = tris.shape[0]
    # each edge k of each cell: key, cell, its circumcentre distance and length
    keys, owner, dd, ll = [], [], [], []
    for k in range(3):
        i, j = (k + 1) % 3, (k + 2) % 3
        keys.append(np.minimum(tris[:, i], tris[:, j]) * mesh.n_vertices + np.maximum(tris[:, i], tris[:, j]))
        owner.append(np.arange(nc))
        dd.append(dist[k])
        ll.append(length[k])
    keys, owner, dd, ll = map(np.concatenate, (keys, owner, dd, ll))
    order = np.argsort(keys, kind="stable")
    ks = keys[order]
    same = ks[1:] == ks[:-1]
    c1, c2 = owner[order][:-1][same], owner[order][1:][same]
    d = dd[order][:-1][same] + dd[order][1:][same]
    w = ll[order][:-1][same] / d
    diag = np.zeros(nc)
    np.add.at(diag, c1, w)
    np.add.at(diag, c2, w)
    rows = np.concatenate([c1, c2, np.arange(nc)])
    cols = np.concatenate([c2, c1, np.arange(nc)])
    vals = np.concatenate([-w, -w, diag])
    K = sp.coo_matrix((vals, (rows, cols)), shape=(nc, nc)).tocsr()
    K.sort_indices()
    Kn = order_n(K, area, n)
    return CellScalarOperator(K=K, Kn=Kn, A=area, n=n, cells=cells, n_cells_total=mesh.n_triangles)


# ------------------------------------------------- Sect. 2.1.2, vertex vectors
@dataclasses.dataclass
class VertexVectorOperator:
    """FE vector Laplacian on vertices, unknowns interleaved ``(u_v, v_v)``
    (east, north) as ``2d, 2d+1``; ``A`` holds the lumped mass per
    component; ``Rvc`` maps a cell velocity field (caller numbering,
    interleaved ``2c, 2c+1``) to the right-hand side."""

    K: sp.csr_matrix
    Kn: sp.csr_matrix
    A: np.ndarray
    n: int
    verts: np.ndarray
    dof_of: np.ndarray
    n_vertices: int
    Rvc: sp.csr_matrix
    n_cells_total: int


def _metric_geometry(mesh, a, b, c):
    """Per triangle: metric factor ``m = tan(theta) / R_e`` with ``theta``
    the latitude of the centroid and ``R_e`` the mean corner radius,
    ``1 / R_e^2``, and the zonal unit vector ``e_E = z x c / |z x c|`` at
    the centroid direction ``c``. Planar meshes: ``m = 0``, ``1/R_e^2 = 0``,
    ``e_E = x``."""
    nf = a.shape[0]
    if mesh.geometry != GEOM_SPHERE:
        return np.zeros(nf), np.zeros(nf), np.tile(np.array([1.0, 0.0, 0.0]), (nf, 1))
    cd = a + b + c
    cd = cd / np.linalg.norm(cd, axis=1, keepdims=True)
    Re = (np.linalg.norm(a, axis=1) + np.linalg.norm(b, axis=1) + np.linalg.norm(c, axis=1)) / 3.0
    coslat = np.hypot(cd[:, 0], cd[:, 1])
    m = cd[:, 2] / (coslat * Re)
    ee = np.stack([-cd[:, 1], cd[:, 0], np.zeros(nf)], axis=1) / coslat[:, None]
    return m, 1.0 / Re ** 2, ee


def vertex_vector_operator(mesh, n: int = 1) -> VertexVectorOperator:
    """The vertex-based FE vector Laplacian of Sect. 2.1.2:
    ``D_2 = [[D~, T], [-T, D~]]`` (l-free) with, over each active triangle
    (P1 basis ``N``, metric factor ``m`` constant on the triangle),

    * ``D~_vv' = int grad N_v . grad N_v' + (R_e^-2 + m^2) N_v N_v'``
      (the scalar stiffness plus a consistent-mass term),
    * ``T_vv' = int m (-N_v' d_x N_v + N_v d_x N_v')``, with ``d_x`` the
      derivative along the zonal unit vector at the centroid; as
      ``d_x N`` is constant on a triangle this is
      ``m A_t / 3 (d_x N_v' - d_x N_v)``.

    ``M_2 = diag(M, M)`` with the lumped (median-dual) mass, order n by
    ``K_n = D_2 (M_2^-1 D_2)^(n-1)``, and the right-hand side
    ``R_vc u_c`` with ``R_vc = int N_v M_c dS = A_c / 3`` for each corner
    ``v`` of an active cell ``c`` (same component to same component).

    Gradients are those of the flat facet: ``grad N_i = n x (P_{i+2} -
    P_{i+1}) / (2 A)`` with ``n`` the facet normal of the corner order.
    """
    K, area, verts, dof_of, tris = cot_stiffness(mesh)
    A = lumped_mass(verts.size, dof_of[tris], area)
    act = active_cells(mesh)
    cells = np.nonzero(act)[0]
    a, b, c = _corner_positions(mesh, tris)
    if a.shape[1] == 2:
        a, b, c = (np.concatenate([p, np.zeros((p.shape[0], 1))], axis=1) for p in (a, b, c))
    m, inv_r2, ee = _metric_geometry(mesh, a, b, c)
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    P = (a, b, c)
    dx = [np.sum(np.cross(nrm, P[(i + 2) % 3] - P[(i + 1) % 3]) * ee, axis=1) / (2.0 * area)
          for i in range(3)]
    idx = dof_of[tris]
    nd = verts.size
    rows, cols, vals = [], [], []
    Kc = K.tocoo()
    for comp in range(2):
        rows.append(2 * Kc.row + comp)
        cols.append(2 * Kc.col + comp)
        vals.append(Kc.data)
    w0 = (inv_r2 + m ** 2) * area / 12.0
    for i in range(3):
        for j in range(3):
            mass_ij = w0 * (2.0 if i == j else 1.0)
            t_ij = m * area / 3.0 * (dx[j] - dx[i])
            for comp in range(2):
                rows.append(2 * idx[:, i] + comp)
                cols.append(2 * idx[:, j] + comp)
                vals.append(mass_ij)
            # T couples east (row) with north (column), -T north with east
            rows += [2 * idx[:, i], 2 * idx[:, i] + 1]
            cols += [2 * idx[:, j] + 1, 2 * idx[:, j]]
            vals += [t_ij, -t_ij]
    D2 = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(2 * nd, 2 * nd)).tocsr()
    D2.sum_duplicates()
    D2.sort_indices()
    A2 = np.repeat(A, 2)
    Kn = order_n(D2, A2, n)
    rr, rc, rv = [], [], []
    for i in range(3):
        for comp in range(2):
            rr.append(2 * idx[:, i] + comp)
            rc.append(2 * cells + comp)
            rv.append(area / 3.0)
    Rvc = sp.coo_matrix((np.concatenate(rv), (np.concatenate(rr), np.concatenate(rc))),
                        shape=(2 * nd, 2 * mesh.n_triangles)).tocsr()
    return VertexVectorOperator(K=D2, Kn=Kn, A=A2, n=n, verts=verts, dof_of=dof_of, n_vertices=mesh.n_vertices,
                                Rvc=Rvc, n_cells_total=mesh.n_triangles)
