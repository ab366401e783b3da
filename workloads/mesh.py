"""Seeded mesh generators.

Two families stand in for the paper's workloads (the FESOM2 meshes are not
available; the data section describes the triangulated rectangular grid):

* ``split_square``: an ``n x n`` lattice with every square cell cut along
  its SW-NE diagonal into two triangles (the construction of the paper's
  data section / Fig. 2), optionally periodic, with each vertex jittered
  by a uniform offset.
* ``icosphere``: the icosahedron refined ``level`` times by 1:4 midpoint
  subdivision and projected onto a sphere of radius ``radius``, with each
  vertex displaced tangentially by a uniform random amount.

``land_mask`` removes vertices inside seeded spherical caps ("blobs").

Only positions and connectivity are produced here; no geometric quantity
that the filter uses (areas, angles, weights) is computed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GEOM_PLANAR = 0
GEOM_PERIODIC = 1
GEOM_SPHERE = 2


@dataclasses.dataclass
class Mesh:
    """A triangle mesh in the layout the C-ABI takes.

    coords : float64 (V, 2) for planar meshes, (V, 3) for the sphere.
    tris   : int32 (F, 3), 0-based vertex ids, counter-clockwise seen from
             above (planar) or from outside (sphere).
    geometry : GEOM_PLANAR, GEOM_PERIODIC or GEOM_SPHERE.
    period : (Px, Py) for GEOM_PERIODIC, else None.
    wet    : uint8 (V,) land mask (1 = ocean) or None (all wet).
    h      : nominal edge length of the unjittered mesh.
    """

    coords: np.ndarray
    tris: np.ndarray
    geometry: int
    period: tuple | None = None
    wet: np.ndarray | None = None
    h: float = 1.0
    radius: float = 0.0
    name: str = ""

    @property
    def n_vertices(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_triangles(self) -> int:
        return int(self.tris.shape[0])

    def with_mask(self, wet: np.ndarray | None) -> "Mesh":
        return dataclasses.replace(self, wet=None if wet is None else np.ascontiguousarray(wet, dtype=np.uint8))


def split_square(n: int, jitter: float = 0.2, periodic: bool = True, seed: int = 1,
                 h: float = 1.0, ny: int | None = None) -> Mesh:
    """``n x ny`` lattice of squares of side ``h``, each split SW-NE.

    Vertex ``(i, j)`` (column i, row j) has id ``i + n*j`` and sits at
    ``h*(i + xi, j + eta)`` with ``xi, eta ~ U(-jitter, jitter)`` drawn from
    ``numpy.random.default_rng(seed)``. The cell with lower-left corner
    ``(i, j)`` gives triangles ``(ij, i+1 j, i+1 j+1)`` and
    ``(ij, i+1 j+1, i j+1)``. With ``periodic`` the lattice wraps with
    period ``(n h, ny h)``; otherwise it has ``(n+1) x (ny+1)`` vertices.
    """
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    nvx, nvy = (n, ny) if periodic else (n + 1, ny + 1)
    jj, ii = np.meshgrid(np.arange(nvy), np.arange(nvx), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    d = rng.uniform(-jitter, jitter, size=(nvx * nvy, 2)) if jitter > 0 else np.zeros((nvx * nvy, 2))
    coords = np.empty((nvx * nvy, 2), dtype=np.float64)
    coords[:, 0] = h * (ii + d[:, 0])
    coords[:, 1] = h * (jj + d[:, 1])

    cj, ci = np.meshgrid(np.arange(ny), np.arange(n), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()

    def vid(i, j):
        if periodic:
            return (i % n) + n * (j % ny)
        return i + nvx * j

    a = vid(ci, cj)
    b = vid(ci + 1, cj)
    c = vid(ci + 1, cj + 1)
    e = vid(ci, cj + 1)
    tris = np.empty((2 * n * ny, 3), dtype=np.int32)
    tris[0::2] = np.stack([a, b, c], axis=1)
    tris[1::2] = np.stack([a, c, e], axis=1)
    geom = GEOM_PERIODIC if periodic else GEOM_PLANAR
    period = (n * h, ny * h) if periodic else None
    name = f"{'periodic' if periodic else 'planar'}-split-square-{n}x{ny}-j{jitter:g}"
    return Mesh(coords=coords, tris=tris, geometry=geom, period=period, h=h, name=name)


def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def _subdivide(v: np.ndarray, f: np.ndarray):
    nv = v.shape[0]
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    key = lo * nv + hi
    uniq, inv = np.unique(key, return_inverse=True)
    ulo = uniq // nv
    uhi = uniq % nv
    mid = v[ulo] + v[uhi]
    mid /= np.linalg.norm(mid, axis=1, keepdims=True)
    nf = f.shape[0]
    m01 = nv + inv[:nf]
    m12 = nv + inv[nf:2 * nf]
    m20 = nv + inv[2 * nf:]
    a, b, c = f[:, 0], f[:, 1], f[:, 2]
    nfaces = np.empty((4 * nf, 3), dtype=np.int64)
    nfaces[0::4] = np.stack([a, m01, m20], axis=1)
    nfaces[1::4] = np.stack([b, m12, m01], axis=1)
    nfaces[2::4] = np.stack([c, m20, m12], axis=1)
    nfaces[3::4] = np.stack([m01, m12, m20], axis=1)
    return np.concatenate([v, mid], axis=0), nfaces


def _mean_edge_length(v: np.ndarray, f: np.ndarray) -> float:
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    key = np.unique(lo * v.shape[0] + hi)
    a = key // v.shape[0]
    b = key % v.shape[0]
    return float(np.linalg.norm(v[a] - v[b], axis=1).mean())


def icosphere(level: int, jitter: float = 0.1, radius: float = 6371.0, seed: int = 1) -> Mesh:
    """Icosahedral sphere mesh with ``10*4**level + 2`` vertices.

    Jitter: every vertex moves by ``jitter*h*(u1 e1 + u2 e2)`` with
    ``u1, u2 ~ U(-1, 1)`` (``default_rng(seed)``), where ``h`` is the mean
    edge (chord) length of the unjittered mesh and ``(e1, e2)`` is the
    tangent basis ``e1 = z x r / |z x r|`` (``e1 = x`` where ``r`` is on
    the polar axis), ``e2 = r x e1``; it is then put back on the sphere.
    """
    v, f = _icosahedron()
    for _ in range(level):
        v, f = _subdivide(v, f)
    h = _mean_edge_length(v, f) * radius
    if jitter > 0:
        rng = np.random.default_rng(seed)
        u = rng.uniform(-1.0, 1.0, size=(v.shape[0], 2))
        z = np.array([0.0, 0.0, 1.0])
        e1 = np.cross(np.broadcast_to(z, v.shape), v)
        n1 = np.linalg.norm(e1, axis=1)
        polar = n1 < 1e-12
        e1[polar] = np.array([1.0, 0.0, 0.0])
        n1[polar] = 1.0
        e1 /= n1[:, None]
        e2 = np.cross(v, e1)
        v = v + (jitter * h / radius) * (u[:, :1] * e1 + u[:, 1:] * e2)
        v /= np.linalg.norm(v, axis=1, keepdims=True)
    coords = np.ascontiguousarray(v * radius)
    tris = np.ascontiguousarray(f.astype(np.int32))
    return Mesh(coords=coords, tris=tris, geometry=GEOM_SPHERE, h=h, radius=radius,
                name=f"icosphere-L{level}-j{jitter:g}")


def land_mask(mesh: Mesh, dry_fraction: float, n_blobs: int = 40, seed: int = 2,
              tol: float = 0.005) -> np.ndarray:
    """Seeded land mask: 1 = wet, 0 = dry.

    ``n_blobs`` cap centres are uniform on the sphere (``default_rng(seed)``)
    with radius factors ``s_b ~ U(0.5, 1.5)``; the common angular radius
    ``rho`` is bisected until the dry share of vertices (inside any cap of
    angular radius ``s_b*rho``) is within ``tol`` of ``dry_fraction``.
    For planar meshes the caps are discs in the plane, with centres uniform
    over the bounding box and ``rho`` a length.
    """
    rng = np.random.default_rng(seed)
    x = mesh.coords
    if mesh.geometry == GEOM_SPHERE:
        cen = rng.normal(size=(n_blobs, 3))
        cen /= np.linalg.norm(cen, axis=1, keepdims=True)
        s = rng.uniform(0.5, 1.5, size=n_blobs)
        xn = x / np.linalg.norm(x, axis=1, keepdims=True)
        # per-vertex: min over blobs of (angle / s_b); dry iff that < rho
        ratio = np.full(x.shape[0], np.inf)
        for b in range(n_blobs):
            ang = np.arccos(np.clip(xn @ cen[b], -1.0, 1.0))
            np.minimum(ratio, ang / s[b], out=ratio)
        lo, hi = 0.0, math.pi
    else:
        lo_xy = x.min(axis=0)
        hi_xy = x.max(axis=0)
        cen = rng.uniform(lo_xy, hi_xy, size=(n_blobs, 2))
        s = rng.uniform(0.5, 1.5, size=n_blobs)
        ratio = np.full(x.shape[0], np.inf)
        for b in range(n_blobs):
            dist = np.linalg.norm(x - cen[b], axis=1)
            np.minimum(ratio, dist / s[b], out=ratio)
        lo, hi = 0.0, float(np.linalg.norm(hi_xy - lo_xy))
    rho = 0.5 * (lo + hi)
    for _ in range(200):
        rho = 0.5 * (lo + hi)
        frac = float(np.mean(ratio < rho))
        if abs(frac - dry_fraction) <= tol:
            break
        if frac < dry_fraction:
            lo = rho
        else:
            hi = rho
    return (ratio >= rho).astype(np.uint8)


def edge_length_scale(mesh: Mesh) -> float:
    """Nominal edge length ``h`` the generator used (unjittered mean edge)."""
    return float(mesh.h)
