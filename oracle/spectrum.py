"""Coarse-graining energy spectrum (oracle, FP64, test-only).

The method's purpose (Sect. 2.1, first paragraph; Sect. 4) is the
distribution of the second moment of a field over scales, obtained from the
coarse-grained fields at a sequence of wavenumbers ``k_l = 1/l``. The paper
prints no formula; the reading used here is

* filtered energy ``E(k) = (1/2) sum_v A_v phi_bar_v^2 / sum_v A_v`` (the
  area-weighted mean; for vectors ``phi_bar^2 = u_bar^2 + v_bar^2``), and
* spectral density ``dE/dk`` by finite differences between neighbouring
  wavenumbers, placed at their geometric mean.
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
