"""Pins of the oracle's spectrum (CPU only)."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _lam(m1, m2, n):
    qx, qy = 2 * np.pi * m1 / n, 2 * np.pi * m2 / n
    return 4 * np.sin(qx / 2) ** 2 + 4 * np.sin(qy / 2) ** 2


@pytest.mark.parametrize("n_order", [1, 2])
def test_single_mode_energy_closed_form(n_order):
    """A single lattice mode a cos(q.x) on the uniform periodic mesh is an
    eigenvector of the filter: E(k) = (1/2)(a^2/2) / (1 + gamma (lam/k^2)^n)^2."""
    N = 32
    m = W.split_square(N, jitter=0.0)
    op = O.scalar_operator(m, n_order)
    a = 1.7
    ks = W.log_scales(1.0, 6)
    for (m1, m2) in ((1, 0), (3, 2), (5, -4)):
        phi = W.planar_mode_field(m, m1, m2, amp=a, phase=0.3)
        out = O.filter_scalar(op, phi, ks, method="dense")
        for j, k in enumerate(ks):
            E = O.energy(op.A, O.to_dofs(op, out[j]))
            ref = 0.5 * (a * a / 2) / (1 + 0.5 * (_lam(m1, m2, N) / k ** 2) ** n_order) ** 2
            assert abs(E / ref - 1) < 1e-12


def test_parseval_over_modes():
    N = 32
    m = W.split_square(N, jitter=0.0)
    op = O.scalar_operator(m, 1)
    modes = [((1, 0), 1.0), ((2, 3), 0.5), ((7, 1), 0.25)]
    phi = sum(W.planar_mode_field(m, a, b, amp=c) for (a, b), c in modes)
    ks = W.log_scales(1.0, 4)
    out = O.filter_scalar(op, phi, ks, method="dense")
    for j, k in enumerate(ks):
        E = O.energy(op.A, O.to_dofs(op, out[j]))
        ref = sum(0.25 * c * c / (1 + 0.5 * _lam(a, b, N) / k ** 2) ** 2 for (a, b), c in modes)
        assert abs(E / ref - 1) < 1e-12


def test_density_of_random_field_is_positive():
    m = W.split_square(32, jitter=0.2)
    op = O.scalar_operator(m, 1)
    phi = W.planar_k3_field(m, 1004)
    ks = W.log_scales(1.0, 8)
    out = O.filter_scalar(op, phi, ks, method="dense")
    E = [O.energy(op.A, O.to_dofs(op, out[j])) for j in range(len(ks))]
    dens, kmid = O.spectrum_density(ks, E)
    assert np.all(dens > 0)
    assert np.all((kmid > ks[:-1]) & (kmid < ks[1:]))
    # energy at the finest scale approaches the unfiltered energy
    assert E[-1] < O.energy(op.A, O.to_dofs(op, phi))
