"""Pins of the oracle's discrete operators against what the paper and the
mathematics fix (CPU only).

Each test would fail for a plausible mistake in ``oracle/operators.py``:
a dropped 1/2, a wrong sign or index, a transposed block, a wrong area
factor or a periodic unwrap error.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W


def _meshes():
    yield "periodic64", W.split_square(64, jitter=0.2)
    yield "planar-patch", W.split_square(12, jitter=0.2, periodic=False, seed=5)
    s = W.icosphere(4, jitter=0.1)
    yield "sphere-L4-mask", s.with_mask(W.land_mask(s, 0.3))


@pytest.mark.parametrize("name,mesh", list(_meshes()))
def test_stiffness_rowsum_symmetry_psd(name, mesh):
    op = O.scalar_operator(mesh, 1)
    K = op.K
    d = K.diagonal()
    # K . 1 = 0: the Laplacian annihilates constants
    assert np.max(np.abs(K @ np.ones(K.shape[0])) / d) < 1e-14
    # symmetry (Sect. 2.1.1: S is symmetric)
    assert abs(K - K.T).max() <= 1e-15 * abs(K).max()
    # positive semidefinite: x^T K x >= 0 and no negative eigenvalue
    rng = np.random.default_rng(0)
    for _ in range(5):
        x = rng.normal(size=K.shape[0])
        assert x @ (K @ x) >= -1e-12 * np.linalg.norm(x) ** 2
    if K.shape[0] <= 5000:
        ev = np.linalg.eigvalsh(K.toarray())
        assert ev.min() >= -1e-12 * ev.max()
    assert np.all(op.A > 0)


def test_uniform_split_square_is_five_point_laplacian():
    """Unjittered split squares: right isosceles triangles give cot-weights
    1 on axis edges, 0 on the diagonals, and A_v = 1 (6 half-unit triangles
    / 3): K is exactly the 5-point Laplacian."""
    n = 16
    m = W.split_square(n, jitter=0.0)
    op = O.scalar_operator(m, 1)
    K = op.K.toarray()
    L5 = np.zeros((n * n, n * n))
    for j in range(n):
        for i in range(n):
            v = i + n * j
            L5[v, v] = 4.0
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                L5[v, ((i + di) % n) + n * ((j + dj) % n)] -= 1.0
    assert np.array_equal(K, L5)
    assert np.max(np.abs(op.A - 1.0)) <= 4e-16
    # the 7-entry pattern of the split-square mesh is kept, diagonals as 0
    assert op.K.nnz == 7 * n * n


def test_linear_precision_interior():
    """P1 stiffness reproduces linear functions: (K x)_v = (K y)_v = 0 at
    interior vertices of a jittered non-periodic patch."""
    m = W.split_square(12, jitter=0.2, periodic=False, seed=5)
    op = O.scalar_operator(m, 1)
    n1 = 13
    ii = op.verts % n1
    jj = op.verts // n1
    interior = (ii > 0) & (ii < n1 - 1) & (jj > 0) & (jj < n1 - 1)
    x = m.coords[op.verts]
    for comp in range(2):
        Kx = op.K @ x[:, comp]
        assert np.max(np.abs(Kx[interior])) < 1e-13
        # but not at the boundary (natural no-flux boundary carries the flux)
        assert np.max(np.abs(Kx[~interior])) > 1e-3


@pytest.mark.parametrize("name,mesh", list(_meshes()))
def test_fv_route_equals_galerkin(name, mesh):
    """Sect. 2.1.1: the finite-volume median-dual treatment leads to the
    same matrix as the P1 Galerkin form."""
    op = O.scalar_operator(mesh, 1)
    Kf = O.fv_stiffness(mesh)
    assert abs(Kf - op.K).max() <= 1e-13 * abs(op.K).max()


def test_mass_totals():
    m = W.split_square(64, jitter=0.2)
    op = O.scalar_operator(m, 1)
    assert abs(op.A.sum() - 64.0 * 64.0) < 1e-9
    s = W.icosphere(4, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    op = O.scalar_operator(s, 1)
    K, area, verts, dof_of, tris = O.cot_stiffness(s)
    assert abs(op.A.sum() - area.sum()) <= 1e-12 * area.sum()
    # flat facets of an unmasked icosphere: a bit less than 4 pi R^2
    s0 = W.icosphere(4, jitter=0.0)
    op0 = O.scalar_operator(s0, 1)
    ratio = op0.A.sum() / (4 * math.pi * s0.radius ** 2)
    assert 0.99 < ratio < 1.0


def test_sphere_rayleigh_quotient_l1_harmonic():
    """z = R cos(colatitude) is an l=1 spherical harmonic: -Lap z = 2 z / R^2.
    On the unjittered icosphere its discrete Rayleigh quotient
    z^T K z / z^T M z equals 2/R^2 exactly (icosahedral symmetry spreads
    facet normals and vertex areas isotropically); on jittered spheres it
    converges to 2/R^2 as the mesh is refined."""
    R = 6371.0
    s = W.icosphere(5, jitter=0.0)
    op = O.scalar_operator(s, 1)
    z = s.coords[:, 2]
    rq = (z @ (op.K @ z)) / (z @ (op.A * z))
    assert abs(rq * R * R / 2 - 1) < 1e-13
    errs = []
    for L in (3, 5):
        sj = W.icosphere(L, jitter=0.1)
        opj = O.scalar_operator(sj, 1)
        zj = sj.coords[:, 2]
        errs.append(abs((zj @ (opj.K @ zj)) / (zj @ (opj.A * zj)) * R * R / 2 - 1))
    assert errs[1] < errs[0] / 10 and errs[1] < 1e-6
    # pointwise M^-1 K z -> 2 z / R^2 on the unjittered mesh (first order)
    e = []
    for L in (3, 4, 5):
        s0 = W.icosphere(L, jitter=0.0)
        o0 = O.scalar_operator(s0, 1)
        z0 = s0.coords[:, 2]
        Lz = (o0.K @ z0) / o0.A
        e.append(np.sqrt(np.sum(o0.A * (Lz - 2 * z0 / R ** 2) ** 2) / np.sum(o0.A * (2 * z0 / R ** 2) ** 2)))
    assert e[1] < 0.6 * e[0] and e[2] < 0.6 * e[1]


def test_order2_operator():
    """Biharmonic K2 = K M^-1 K (Sect. 2.1.1, Eq. 5): symmetric,
    annihilates constants, equals the composed operator."""
    s = W.icosphere(4, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    op = O.scalar_operator(s, 2)
    K2 = op.Kn
    assert abs(K2 - K2.T).max() <= 1e-15 * abs(K2).max()
    assert np.max(np.abs(K2 @ np.ones(K2.shape[0]))) <= 1e-14 * abs(K2).max()
    x = np.random.default_rng(1).normal(size=K2.shape[0])
    y = op.K @ ((op.K @ x) / op.A)
    assert np.linalg.norm(K2 @ x - y) <= 1e-14 * np.linalg.norm(y)
    # 2-ring pattern: up to 19 entries per row on a valence-6 mesh
    assert np.diff(K2.indptr).max() <= 19


def test_order4_operator():
    """K4 = K (M^-1 K)^3 (Sect. 2.1.1 at n = 4): symmetric, annihilates
    constants, equals four applications of the Laplacian form, and reaches
    the 4-ring (61 entries a row on a valence-6 mesh)."""
    s = W.icosphere(3, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    op = O.scalar_operator(s, 4)
    K4 = op.Kn
    assert abs(K4 - K4.T).max() <= 1e-14 * abs(K4).max()
    assert np.max(np.abs(K4 @ np.ones(K4.shape[0]))) <= 1e-13 * abs(K4).max()
    x = np.random.default_rng(2).normal(size=K4.shape[0])
    y = x
    for r in range(4):
        y = op.K @ y if r == 3 else (op.K @ y) / op.A
    assert np.linalg.norm(K4 @ x - y) <= 1e-13 * np.linalg.norm(y)
    assert np.diff(K4.indptr).max() <= 61


def test_dofs_exclude_dry_and_orphans():
    s = W.icosphere(3, jitter=0.1)
    wet = W.land_mask(s, 0.4, seed=3)
    s = s.with_mask(wet)
    op = O.scalar_operator(s, 1)
    act = O.active_cells(s)
    used = np.zeros(s.n_vertices, bool)
    used[s.tris[act].ravel()] = True
    assert np.array_equal(np.sort(op.verts), np.nonzero(used)[0])
    assert np.all(wet[op.verts] == 1)
