"""Pins of the oracle's cell-vector operator (Eq. 7), CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.solve import relative_l2

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_symmetric_psd_sphere():
    """Sect. 2.1.2: operator (7) is symmetric positive semidefinite."""
    s = W.icosphere(3, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    vo = O.vector_operator(s, 1)
    K = vo.K.toarray()
    assert np.max(np.abs(K - K.T)) == 0.0
    ev = np.linalg.eigvalsh(K)
    assert ev.min() >= -1e-12 * ev.max()


def test_planar_decouples():
    """On a plane the unit vectors do not turn: no u-v coupling, and both
    components see the same scalar cell Laplacian."""
    m = W.split_square(10, jitter=0.2)
    vo = O.vector_operator(m, 1, stencil_A=1.5)
    K = vo.K.toarray()
    assert np.max(np.abs(K[0::2, 1::2])) == 0.0
    assert np.array_equal(K[0::2, 0::2], K[1::2, 1::2])
    u = W.planar_k3_velocity(m, 1, 2)
    ks = W.log_scales(1.0, 3)
    out = O.filter_vector(vo, u.reshape(-1), ks, method="dense")
    # filtering a field with v = 0 leaves v = 0
    u0 = u.copy()
    u0[:, 1] = 0
    out0 = O.filter_vector(vo, u0.reshape(-1), ks, method="dense")
    assert np.max(np.abs(out0[:, :, 1])) == 0.0
    assert relative_l2(out0[:, :, 0], out[:, :, 0]) < 1e-13


def _bloch_lower(vo, mesh, cells, q):
    """Lower eigenvalue of the Bloch symbol of M^-1 K built from the
    assembled stencil of two sublattice cells."""
    K = vo.K.tocsr()
    cen = _centroids(mesh)
    H = np.zeros((2, 2), dtype=complex)
    for a, ca in enumerate(cells):
        row = K.getrow(2 * ca)
        for col, val in zip(row.indices, row.data):
            if col % 2:
                continue
            cb = col // 2
            d = cen[cb] - cen[ca]
            p = np.asarray(mesh.period)
            d = d - p * np.round(d / p)
            b = 0 if (cb % 2) == (cells[0] % 2) else 1
            H[a, b] += val * np.exp(1j * (q @ d))
    H /= vo.A[2 * cells[0]]
    return np.linalg.eigvalsh(H).min()


def _centroids(mesh):
    x = mesh.coords
    t = mesh.tris
    a = x[t[:, 0]]
    p = np.asarray(mesh.period)
    b = a + (x[t[:, 1]] - a) - p * np.round((x[t[:, 1]] - a) / p)
    c = a + (x[t[:, 2]] - a) - p * np.round((x[t[:, 2]] - a) / p)
    return (a + b + c) / 3.0


def test_split_square_continuum_limit():
    """Sect. 2.1.2: on squares split into two triangles, A = 3/2 gives
    -dxx - dyy +/- dxy; for the SW-NE split the symbol of the smooth branch
    is qx^2 + qy^2 + qx qy."""
    A = GOLD["cell_stencil_A_split_squares"]["value"]
    m = W.split_square(8, jitter=0.0)
    vo = O.vector_operator(m, 1, stencil_A=A)
    for t in np.linspace(0, np.pi, 7):
        q = 0.01 * np.array([math.cos(t), math.sin(t)])
        lam = _bloch_lower(vo, m, [0, 1], q)
        ref = q[0] ** 2 + q[1] ** 2 + q[0] * q[1]
        assert abs(lam / ref - 1) < 1e-3


def _equilateral_periodic(n, rows):
    """Periodic lattice of equilateral triangles (unit edge), ``rows`` even;
    even triangle ids point up, odd ids point down (the two sublattices)."""
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


def test_equilateral_continuum_limit():
    """Sect. 2.1.2: A = sqrt(3) on equilateral triangles gives -Laplacian."""
    A = GOLD["cell_stencil_A_equilateral"]["value"]
    m = _equilateral_periodic(6, 6)
    vo = O.vector_operator(m, 1, stencil_A=A)
    assert np.allclose(vo.K.diagonal(), 3 * A)
    for t in np.linspace(0, np.pi, 5):
        q = 0.01 * np.array([math.cos(t), math.sin(t)])
        lam = _bloch_lower(vo, m, [0, 1], q)
        assert abs(lam / (q @ q) - 1) < 1e-3


def _frames(mesh):
    x = mesh.coords
    t = mesh.tris
    c = x[t[:, 0]] + x[t[:, 1]] + x[t[:, 2]]
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    ee = np.cross(np.array([0.0, 0.0, 1.0]), c)
    ee /= np.linalg.norm(ee, axis=1, keepdims=True)
    return ee, np.cross(c, ee)


def test_frame_independence_under_rotation():
    """The metric treatment must not depend on where the poles are: rotate
    the mesh and the 3-D velocity rigidly, filter, and compare with the
    rotated filtered field."""
    s = W.icosphere(3, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    u = W.sphere_k3_velocity(s, 11, 12, n_waves=128)
    ks = W.log_scales(s.h, 3)
    vo = O.vector_operator(s, 1)
    out = O.filter_vector(vo, u.reshape(-1), ks, method="dense")
    ee, en = _frames(s)
    u3 = u[:, :1] * ee + u[:, 1:] * en
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    sr = W.Mesh(coords=s.coords @ Q.T, tris=s.tris, geometry=W.GEOM_SPHERE, wet=s.wet, h=s.h, radius=s.radius)
    eer, enr = _frames(sr)
    ur3 = u3 @ Q.T
    ur = np.stack([np.sum(ur3 * eer, 1), np.sum(ur3 * enr, 1)], 1)
    vr = O.vector_operator(sr, 1)
    outr = O.filter_vector(vr, ur.reshape(-1), ks, method="dense")
    for j in range(len(ks)):
        a3 = out[j][:, :1] * ee + out[j][:, 1:] * en
        b3 = outr[j][:, :1] * eer + outr[j][:, 1:] * enr
        assert relative_l2(b3, a3 @ Q.T) < 1e-12


def test_vector_invariants():
    s = W.icosphere(4, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    u = W.sphere_k3_velocity(s, 21, 22, n_waves=256)
    vo = O.vector_operator(s, 1)
    ks = W.log_scales(s.h, 4)
    out = O.filter_vector(vo, u.reshape(-1), ks)
    x0 = O.to_dofs(vo, u.reshape(-1))
    e0 = vo.A @ (x0 * x0)
    prev = 0.0
    for j in range(len(ks)):
        x = O.to_dofs(vo, out[j].reshape(-1))
        e = vo.A @ (x * x)
        assert prev * (1 - 1e-14) <= e <= e0 * (1 + 1e-14)
        prev = e
