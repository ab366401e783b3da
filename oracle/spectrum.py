"""Coarse-graining energy spectrum (oracle, FP64, test-only).

The method's purpose (Sect. 2.1, first paragraph; Sect. 4) is the
distribution of the second moment of a field over scales, obtained from the
coarse-grained fields at a sequence of wavenumbers ``k_l = 1/l``. The paper
prints no formula; the reading used here is

* filtered energy ``E(k) = (1/2) sum_v A_v phi_bar_v^2 / sum_v A_v`` (the
  area-weighted mean; for vectors ``phi_bar^2 = u_bar^2 + v_bar^2``), and
* spectral density ``dE/dk`` by finite differences between neighbouring
  wavenumbers, placed at their geometric mean.

The theoretical spectra of the "Some comments" section (Fig. 8) filter a
prescribed Fourier spectrum with the analytic transfer function of the
implicit filter built on the 1-D discrete Laplacian: a Fourier mode of
wavenumber q is an eigenvector of the filter on a uniform periodic grid,
damped by ``G = 1 / (1 + gamma (lam(q) / k^2)^n)`` with the discrete symbol
``lam(q) = 4 sin^2(q h / 2) / h^2``, so its filtered energy is ``G^2``
times its energy.
"""
from __future__ import annotations

import numpy as np


def energy(A: np.ndarray, xbar: np.ndarray) -> float:
    """``(1/2) sum A x^2 / sum A`` over dofs; ``A`` and ``xbar`` share the
    dof layout (for vectors ``A`` is repeated per component and the sum
    is over cells, hence the division by the per-cell area sum)."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(xbar, dtype=np.float64)
    return float(0.5 * np.sum(A * x * x) / np.sum(A))


def spectrum_density(ks, E):
    """Finite-difference density ``(E_{j+1} - E_j) / (k_{j+1} - k_j)`` at
    ``k_mid = sqrt(k_j k_{j+1})``; ``ks`` ascending."""
    ks = np.asarray(ks, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    dens = (E[1:] - E[:-1]) / (ks[1:] - ks[:-1])
    kmid = np.sqrt(ks[1:] * ks[:-1])
    return dens, kmid


def discrete_symbol(q, h: float = 1.0):
    """Fourier symbol of the 1-D second-difference Laplacian (-D2) on a
    grid of spacing h: ``4 sin^2(q h / 2) / h^2``."""
    q = np.asarray(q, dtype=np.float64)
    return 4.0 * np.sin(0.5 * q * h) ** 2 / (h * h)


def filtered_energy_of_modes(q, E_q, ks, n: int, gamma: float = 0.5, h: float = 1.0):
    """Filtered energy ``E(k) = sum_q E_q / (1 + gamma (lam(q)/k^2)^n)^2``
    of a field whose Fourier modes q carry energies E_q, at each k."""
    lam = discrete_symbol(q, h)
    E_q = np.asarray(E_q, dtype=np.float64)
    out = []
    for k in np.asarray(ks, dtype=np.float64):
        G = 1.0 / (1.0 + gamma * (lam / (k * k)) ** n)
        out.append(float(np.sum(E_q * G * G)))
    return np.array(out)


def fig8_modes(N: int, h: float = 1.0, k_star_over_kmin: float = 30.0):
    """The prescribed spectrum of Fig. 8, ``E_q ~ q^-2 / (1 + (q/k*)^2)``
    with ``k* = 30 k_min``, on the modes q = 2 pi m / (N h), m = 1 .. N/2 - 1
    of a periodic grid of N points (k_min = 2 pi / (N h), the domain
    wavenumber; the Nyquist mode is left out). Returns (q, E_q)."""
    m = np.arange(1, N // 2)
    q = 2.0 * np.pi * m / (N * h)
    k_star = k_star_over_kmin * 2.0 * np.pi / (N * h)
    E_q = q ** -2.0 / (1.0 + (q / k_star) ** 2)
    return q, E_q
