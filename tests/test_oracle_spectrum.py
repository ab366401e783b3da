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


def _fig8_field(mesh, N, seed=5):
    """The Fig. 8 spectrum as a field of 1-D modes along x on the uniform
    periodic split square (mode m carries energy E_m = a_m^2 / 4)."""
    q, E = O.fig8_modes(N)
    rng = np.random.default_rng(seed)
    phases = rng.uniform(0, 2 * np.pi, q.size)
    phi = sum(W.planar_mode_field(mesh, m, 0, amp=2 * np.sqrt(e), phase=t)
              for m, e, t in zip(range(1, N // 2), E, phases))
    return phi, q, E


@pytest.mark.parametrize("n_order", [1, 2])
def test_fig8_closed_form_matches_the_assembled_filter(n_order):
    """"Some comments" section (Fig. 8): the theoretical spectrum is the
    prescribed one damped by the analytic transfer function of the filter
    built on the discrete Laplacian symbol. On the uniform periodic split
    square, modes along x see exactly that symbol (the assembled P1
    stiffness is the 5-point Laplacian there), so the filtered energy of
    the assembled filter equals the closed form."""
    N = 32
    m = W.split_square(N, jitter=0.0)
    op = O.scalar_operator(m, n_order)
    phi, q, E = _fig8_field(m, N)
    ks = W.log_scales(1.0, 5)
    out = O.filter_scalar(op, phi, ks, method="dense")
    got = [O.energy(op.A, O.to_dofs(op, out[j])) for j in range(len(ks))]
    ref = O.filtered_energy_of_modes(q, E, ks, n_order)
    assert np.max(np.abs(np.array(got) / ref - 1)) < 1e-11
    # unfiltered energy: Parseval over the prescribed modes
    assert abs(O.energy(op.A, O.to_dofs(op, phi)) / E.sum() - 1) < 1e-12


def test_fig8_four_harmonic_closed_form_matches_a_dense_filter():
    """n = 4 (the four-harmonic curve of Fig. 8) from the closed form against
    the filter applied as a dense matrix power on a 1-D periodic grid."""
    N = 64
    q, E = O.fig8_modes(N)
    x = np.arange(N, dtype=np.float64)
    rng = np.random.default_rng(9)
    phi = sum(2 * np.sqrt(e) * np.cos(qq * x + t) for qq, e, t in zip(q, E, rng.uniform(0, 2 * np.pi, q.size)))
    L = 2 * np.eye(N) - np.roll(np.eye(N), 1, axis=1) - np.roll(np.eye(N), -1, axis=1)
    # k not too small: the dense solve's condition number is (4 / k^2)^4
    for k in (0.6, 1.0, 2.0):
        S = np.eye(N) + 0.5 * np.linalg.matrix_power(L / k ** 2, 4)
        fbar = np.linalg.solve(S, phi)
        got = 0.5 * np.mean(fbar ** 2)
        ref = O.filtered_energy_of_modes(q, E, [k], 4)[0]
        assert abs(got / ref - 1) < 1e-10


def test_fig8_higher_orders_follow_the_steep_slope():
    """The qualitative content of Fig. 8: where the prescribed spectrum falls
    as k^-4 (k > k*), the Laplacian filter's spectrum is flatter than k^-3,
    and the biharmonic and four-harmonic filters come successively closer to
    the prescribed spectrum."""
    N = 2048
    q, E = O.fig8_modes(N)
    dq = q[1] - q[0]
    k_star = 30 * 2 * np.pi / N
    ks = np.exp(np.linspace(np.log(4 * np.pi / N), np.log(0.9 * np.pi), 60))
    errs, slopes = {}, {}
    for n in (1, 2, 4):
        dens, km = O.spectrum_density(ks, O.filtered_energy_of_modes(q, E, ks, n))
        sel = (km > 4 * k_star) & (km < 0.5 * np.pi)
        true = np.interp(km[sel], q, E / dq)
        errs[n] = np.sqrt(np.mean(np.log(dens[sel] / true) ** 2))
        slopes[n] = np.diff(np.log(dens[sel])) / np.diff(np.log(km[sel]))
    assert np.all(slopes[1] > -3.0)
    assert errs[4] < errs[2] < errs[1]
    assert errs[4] < 0.5


def _dE_dk(q, E_q, ks, n, gamma=0.5):
    """Analytic k-derivative of filtered_energy_of_modes: with
    G = 1 / (1 + gamma (lam/k^2)^n), dG/dk = G^2 2 n gamma (lam/k^2)^n / k,
    so dE/dk = sum_q E_q 4 n gamma (lam/k^2)^n G^3 / k."""
    lam = O.discrete_symbol(q)
    out = []
    for k in ks:
        t = gamma * (lam / (k * k)) ** n
        G = 1.0 / (1.0 + t)
        out.append(float(np.sum(E_q * 4.0 * n * t * G ** 3 / k)))
    return np.array(out)


def _density_pins(density, n_order):
    """The checks of test_density_is_the_k_derivative_of_the_fig8_energy on
    a density function; returns the names of the failed ones."""
    N = 2048
    q, E = O.fig8_modes(N)
    ks = np.exp(np.arange(np.log(4 * np.pi / N), np.log(0.5 * np.pi), np.log1p(1e-3)))[::37]
    fine = np.exp(np.log(ks)[:, None] + np.array([0.0, np.log1p(1e-3)])[None, :]).ravel()
    Ef = O.filtered_energy_of_modes(q, E, fine, n_order)
    dens, km = density(fine, Ef)
    dens, km = dens[::2], km[::2]  # the pairs (k, k (1 + 1e-3))
    ref = _dE_dk(q, E, km, n_order)
    sel = ref > 1e-12 * ref.max()
    failed = []
    if not np.max(np.abs(dens[sel] / ref[sel] - 1)) < 1e-4:
        failed.append("derivative")
    kc = np.exp(np.linspace(np.log(4 * np.pi / N), np.log(0.9 * np.pi), 25))
    Ec = O.filtered_energy_of_modes(q, E, kc, n_order)
    dc, kmc = density(kc, Ec)
    if not abs(np.sum(dc * np.diff(kc)) / (Ec[-1] - Ec[0]) - 1) < 1e-12:
        failed.append("telescoping")
    if not np.allclose(kmc * kmc, kc[:-1] * kc[1:], rtol=1e-14, atol=0):
        failed.append("midpoint")
    return failed


def _mutant_arithmetic_mid(ks, E):
    d, _ = O.spectrum_density(ks, E)
    return d, 0.5 * (ks[1:] + ks[:-1])


def _mutant_step(ks, E):
    d, km = O.spectrum_density(ks, E)
    return d / 1.6, km


def _mutant_left_point(ks, E):
    d, _ = O.spectrum_density(ks, E)
    return d, np.asarray(ks)[:-1]


@pytest.mark.parametrize("n_order", [1, 2, 4])
def test_density_pins_reject_planted_mistakes(n_order):
    """The density pins hold for the oracle and fail for the oracle with a
    planted mistake: the arithmetic instead of the geometric midpoint, a
    step scaled by 1.6, or the difference placed at the left wavenumber."""
    assert _density_pins(O.spectrum_density, n_order) == []
    assert "midpoint" in _density_pins(_mutant_arithmetic_mid, n_order)
    assert _density_pins(_mutant_step, n_order)
    assert "derivative" in _density_pins(_mutant_left_point, n_order)


@pytest.mark.parametrize("n_order", [1, 2, 4])
def test_density_is_the_k_derivative_of_the_fig8_energy(n_order):
    """spectrum_density on the Fig. 8 construction ("Some comments"
    section) at fine, log-spaced k (ratio 1 + 1e-3 between neighbours) is
    the analytic derivative dE/dk at k_mid: a central difference, so the
    error is O((dk/k)^2) ~ 1e-6, where a difference off by one index or a
    step scaled wrongly is off by ~1e-3 or more. Summed over the steps the
    density gives back the energy difference (telescoping), and k_mid is the
    geometric mean of the two wavenumbers."""
    N = 2048
    q, E = O.fig8_modes(N)
    ks = np.exp(np.arange(np.log(4 * np.pi / N), np.log(0.5 * np.pi), np.log1p(1e-3)))[::37]
    fine = np.exp(np.log(ks)[:, None] + np.array([0.0, np.log1p(1e-3)])[None, :]).ravel()
    Ef = O.filtered_energy_of_modes(q, E, fine, n_order)
    dens, km = O.spectrum_density(fine, Ef)
    dens, km = dens[::2], km[::2]  # the pairs (k, k (1 + 1e-3))
    ref = _dE_dk(q, E, km, n_order)
    sel = ref > 1e-12 * ref.max()
    assert np.max(np.abs(dens[sel] / ref[sel] - 1)) < 1e-4
    # telescoping over a coarse list and the geometric midpoint
    kc = np.exp(np.linspace(np.log(4 * np.pi / N), np.log(0.9 * np.pi), 25))
    Ec = O.filtered_energy_of_modes(q, E, kc, n_order)
    dc, kmc = O.spectrum_density(kc, Ec)
    assert abs(np.sum(dc * np.diff(kc)) / (Ec[-1] - Ec[0]) - 1) < 1e-12
    assert np.allclose(kmc * kmc, kc[:-1] * kc[1:], rtol=1e-14, atol=0)
