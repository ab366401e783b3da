"""Seeded random fields with an isotropic k^-3 energy spectrum.

* Planar periodic meshes: a sum over the lattice modes of the period,
  ``q = 2*pi*(m1/Px, m2/Py)``, ``0 < |q| <= pi/h``, with Gaussian cosine and
  sine amplitudes of standard deviation ``|q|^-2`` (so the shell energy
  ``2*pi*|q|*|q|^-4`` falls as ``|q|^-3``), evaluated exactly at the
  (jittered) vertex positions.
* Spheres: ``n_waves`` 3-D plane waves ``a_j cos(q_j . x + theta_j)`` with
  ``|q_j|`` log-uniform on ``[2/R, pi/h]``, direction uniform on the unit
  sphere and phase uniform, ``a_j ~ |q_j|^-1`` (energy per log-wavenumber
  ``~ |q|^-2``, i.e. ``E(k) ~ k^-3``).

Every field is scaled to unit RMS over the wet vertices (or cells). The
sphere generator runs in torch so that large fields can be drawn on the
device; the random draws themselves come from numpy, so the values do not
depend on the device beyond the last bits of ``cos``.
"""
from __future__ import annotations

import math

import numpy as np

from .mesh import GEOM_PERIODIC, GEOM_SPHERE, Mesh


def log_scales(h: float, n_scales: int, lam_max_cells: float = 32.0, lam_min_cells: float = 2.0) -> np.ndarray:
    """Ascending wavenumbers ``k_j = 2*pi/lambda_j`` with wavelengths
    log-spaced from ``lam_max_cells*h`` down to ``lam_min_cells*h``."""
    if n_scales == 1:
        lam = np.array([lam_max_cells * h])
    else:
        t = np.arange(n_scales) / (n_scales - 1)
        lam = lam_max_cells * h * (lam_min_cells / lam_max_cells) ** t
    return 2.0 * math.pi / lam


def _planar_modes(mesh: Mesh):
    assert mesh.geometry == GEOM_PERIODIC, "planar k^-3 fields need a periodic mesh"
    px, py = mesh.period
    mx = int(round(px / mesh.h))
    my = int(round(py / mesh.h))
    m1, m2 = np.meshgrid(np.arange(-mx // 2, mx // 2 + 1), np.arange(0, my // 2 + 1), indexing="ij")
    m1 = m1.ravel()
    m2 = m2.ravel()
    half = (m2 > 0) | ((m2 == 0) & (m1 > 0))
    m1 = m1[half]
    m2 = m2[half]
    qx = 2.0 * math.pi * m1 / px
    qy = 2.0 * math.pi * m2 / py
    qn = np.hypot(qx, qy)
    keep = (qn > 0) & (qn <= math.pi / mesh.h + 1e-12)
    return qx[keep], qy[keep], qn[keep]


def _unit_rms(phi: np.ndarray, wet: np.ndarray | None) -> np.ndarray:
    sel = phi if wet is None else phi[wet.astype(bool)]
    rms = math.sqrt(float(np.mean(sel * sel)))
    out = phi / rms
    if wet is not None:
        out = np.where(wet.astype(bool), out, 0.0)
    return out


def planar_k3_field(mesh: Mesh, seed: int) -> np.ndarray:
    """k^-3 Gaussian random field on a periodic planar mesh (float64, V)."""
    rng = np.random.default_rng(seed)
    qx, qy, qn = _planar_modes(mesh)
    a = rng.normal(size=qn.size) * qn ** -2.0
    b = rng.normal(size=qn.size) * qn ** -2.0
    x = mesh.coords
    phase = np.outer(x[:, 0], qx) + np.outer(x[:, 1], qy)
    phi = np.cos(phase) @ a + np.sin(phase) @ b
    return _unit_rms(phi, mesh.wet)


def planar_k3_velocity(mesh: Mesh, seed_psi: int, seed_chi: int, div_frac: float = 0.1,
                       points: np.ndarray | None = None) -> np.ndarray:
    """Velocity ``(-d_y psi, d_x psi) + grad chi`` at ``points`` (default:
    the triangle centroids, minimum-image), with ``chi`` scaled so its RMS
    speed is ``div_frac`` of the rotational part. Returns (P, 2)."""
    if points is None:
        points = _planar_centroids(mesh)
    qx, qy, qn = _planar_modes(mesh)

    def grad(seed):
        rng = np.random.default_rng(seed)
        a = rng.normal(size=qn.size) * qn ** -2.0
        b = rng.normal(size=qn.size) * qn ** -2.0
        ph = np.outer(points[:, 0], qx) + np.outer(points[:, 1], qy)
        d = -np.sin(ph) * a + np.cos(ph) * b  # derivative of the phase sum
        return np.stack([d @ qx, d @ qy], axis=1)

    gp = grad(seed_psi)
    gc = grad(seed_chi)
    rot = np.stack([-gp[:, 1], gp[:, 0]], axis=1)
    rms_rot = math.sqrt(float(np.mean(np.sum(rot * rot, axis=1))))
    rms_div = math.sqrt(float(np.mean(np.sum(gc * gc, axis=1))))
    u = rot + (div_frac * rms_rot / rms_div) * gc
    return u / rms_rot


def _planar_centroids(mesh: Mesh) -> np.ndarray:
    x = mesh.coords
    t = mesh.tris
    a = x[t[:, 0]]
    b = x[t[:, 1]]
    c = x[t[:, 2]]
    if mesh.period is not None:
        p = np.asarray(mesh.period)
        b = a + (b - a) - p * np.round((b - a) / p)
        c = a + (c - a) - p * np.round((c - a) / p)
    return (a + b + c) / 3.0


def planar_mode_field(mesh: Mesh, m1: int, m2: int, amp: float = 1.0, phase: float = 0.0) -> np.ndarray:
    """Single lattice mode ``amp*cos(q.x + phase)``, ``q = 2*pi*(m1/Px, m2/Py)``."""
    px, py = mesh.period
    q = np.array([2.0 * math.pi * m1 / px, 2.0 * math.pi * m2 / py])
    return amp * np.cos(mesh.coords @ q + phase)


def _sphere_waves(seed: int, radius: float, h: float, n_waves: int):
    rng = np.random.default_rng(seed)
    kmin = 2.0 / radius
    kmax = math.pi / h
    lk = rng.uniform(math.log(kmin), math.log(kmax), size=n_waves)
    kn = np.exp(lk)
    d = rng.normal(size=(n_waves, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    q = d * kn[:, None]
    theta = rng.uniform(0.0, 2.0 * math.pi, size=n_waves)
    dlnk = (math.log(kmax) - math.log(kmin)) / n_waves
    amp = np.sqrt(2.0 * dlnk) / kn
    return q, theta, amp


def _eval_waves(points, q, theta, amp, device, grad: bool = False, chunk: int = 1 << 18):
    import torch

    dev = torch.device(device if device is not None else "cpu")
    qt = torch.as_tensor(q, dtype=torch.float64, device=dev)
    th = torch.as_tensor(theta, dtype=torch.float64, device=dev)
    am = torch.as_tensor(amp, dtype=torch.float64, device=dev)
    pts = torch.as_tensor(np.ascontiguousarray(points), dtype=torch.float64, device=dev)
    n = pts.shape[0]
    out = torch.empty((n, 3) if grad else (n,), dtype=torch.float64, device=dev)
    for s in range(0, n, chunk):
        ph = pts[s:s + chunk] @ qt.T + th
        if grad:
            out[s:s + chunk] = (-torch.sin(ph) * am) @ qt
        else:
            out[s:s + chunk] = torch.cos(ph) @ am
    return out.cpu().numpy()


def sphere_k3_field(mesh: Mesh, seed: int, n_waves: int = 1024, device=None) -> np.ndarray:
    """k^-3 random field at the vertices of a sphere mesh (float64, V)."""
    assert mesh.geometry == GEOM_SPHERE
    q, th, am = _sphere_waves(seed, mesh.radius, mesh.h, n_waves)
    phi = _eval_waves(mesh.coords, q, th, am, device)
    return _unit_rms(phi, mesh.wet)


def sphere_k3_velocity(mesh: Mesh, seed_psi: int, seed_chi: int, div_frac: float = 0.1,
                       n_waves: int = 1024, device=None) -> np.ndarray:
    """Velocity on triangle cells of a sphere mesh, (F, 2) = (east, north).

    ``u = r x grad psi + grad chi`` (tangential gradients of two independent
    k^-3 fields, evaluated analytically at the centroid direction ``c`` put
    on the sphere), with ``chi`` scaled so its RMS speed is ``div_frac`` of
    the rotational part. Components are taken on ``e_E = z x c / |z x c|``,
    ``e_N = c x e_E``. Cells with a dry vertex are set to zero.
    """
    assert mesh.geometry == GEOM_SPHERE
    x = mesh.coords
    t = mesh.tris
    cen = x[t[:, 0]] + x[t[:, 1]] + x[t[:, 2]]
    c = cen / np.linalg.norm(cen, axis=1, keepdims=True)
    pts = c * mesh.radius

    def tgrad(seed):
        q, th, am = _sphere_waves(seed, mesh.radius, mesh.h, n_waves)
        g = _eval_waves(pts, q, th, am, device, grad=True)
        return g - np.sum(g * c, axis=1, keepdims=True) * c

    gp = tgrad(seed_psi)
    gc = tgrad(seed_chi)
    rot = np.cross(c, gp)
    active = np.ones(t.shape[0], dtype=bool)
    if mesh.wet is not None:
        w = mesh.wet.astype(bool)
        active = w[t[:, 0]] & w[t[:, 1]] & w[t[:, 2]]
    rms_rot = math.sqrt(float(np.mean(np.sum(rot[active] ** 2, axis=1))))
    rms_div = math.sqrt(float(np.mean(np.sum(gc[active] ** 2, axis=1))))
    u3 = (rot + (div_frac * rms_rot / rms_div) * gc) / rms_rot
    z = np.array([0.0, 0.0, 1.0])
    ee = np.cross(np.broadcast_to(z, c.shape), c)
    ee /= np.linalg.norm(ee, axis=1, keepdims=True)
    en = np.cross(c, ee)
    out = np.stack([np.sum(u3 * ee, axis=1), np.sum(u3 * en, axis=1)], axis=1)
    out[~active] = 0.0
    return np.ascontiguousarray(out)
