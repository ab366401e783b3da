"""Pins of the oracle's filter solve (CPU only): the closed-form Fourier
multiplier on a uniform periodic mesh, filter invariants, and the CG path
against dense Cholesky / LAPACK."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.solve import relative_l2, residual_bound


def _fourier_filter(phi_grid, k, gamma, n):
    """Closed form on the unjittered periodic split-square lattice (h = 1):
    K is the 5-point Laplacian with symbol lam(q) = 4 sin^2(qx/2) +
    4 sin^2(qy/2), M = I, and K_n has symbol lam^n, so each Fourier mode
    is multiplied by 1 / (1 + gamma (lam / k^2)^n)."""
    ny, nx = phi_grid.shape
    qx = 2 * np.pi * np.fft.fftfreq(nx)
    qy = 2 * np.pi * np.fft.fftfreq(ny)
    QX, QY = np.meshgrid(qx, qy)
    lam = 4 * np.sin(QX / 2) ** 2 + 4 * np.sin(QY / 2) ** 2
    mult = 1.0 / (1.0 + gamma * (lam / k ** 2) ** n)
    return np.real(np.fft.ifft2(np.fft.fft2(phi_grid) * mult))


@pytest.mark.parametrize("n", [1, 2])
@pytest.mark.parametrize("gamma", [0.5, 1.0])
def test_closed_form_fourier_multiplier(n, gamma):
    N = 32
    m = W.split_square(N, jitter=0.0)
    op = O.scalar_operator(m, n)
    phi = W.planar_k3_field(m, 1000)
    ks = W.log_scales(1.0, 5)
    for method in ("dense", "cg"):
        out = O.filter_scalar(op, phi, ks, gamma=gamma, method=method)
        for j, k in enumerate(ks):
            ref = _fourier_filter(phi.reshape(N, N), k, gamma, n).ravel()
            assert relative_l2(out[j], ref) < 1e-12, (method, j)


@pytest.mark.parametrize("n", [3, 4])
def test_closed_form_fourier_multiplier_higher_orders(n):
    """Orders 3 and 4 (K_n = K (M^-1 K)^(n-1), Sect. 2.1.1; n = 4 is the
    highest order of Fig. 8): on the uniform periodic split square the
    filter is the multiplier 1 / (1 + gamma (lambda / k^2)^n). Scales stop at
    8 cells, where the condition number (~1e4) leaves the direct solves
    accurate to 1e-12."""
    N = 32
    m = W.split_square(N, jitter=0.0)
    op = O.scalar_operator(m, n)
    phi = W.planar_k3_field(m, 1000)
    ks = W.log_scales(1.0, 4, lam_max_cells=8.0)
    for method in ("dense", "direct"):
        out = O.filter_scalar(op, phi, ks, method=method)
        for j, k in enumerate(ks):
            ref = _fourier_filter(phi.reshape(N, N), k, 0.5, n).ravel()
            assert relative_l2(out[j], ref) < 1e-12, (method, j)


def test_cg_matches_dense_and_lapack_c1():
    """Plain FP64 configuration: 64x64 periodic split square, jitter 0.2,
    n = 1, eight scales from 32 to 2 cells: CG (from x0 = phi) equals the
    dense Cholesky solve and LAPACK's general solve."""
    m = W.split_square(64, jitter=0.2)
    op = O.scalar_operator(m, 1)
    phi = W.planar_k3_field(m, 1000)
    ks = W.log_scales(1.0, 8)
    dense = O.filter_scalar(op, phi, ks, method="dense")
    cg = O.filter_scalar(op, phi, ks, method="cg")
    for j, k in enumerate(ks):
        assert relative_l2(cg[j], dense[j]) < 1e-12
    S = O.system_matrix(op, ks[0])
    lap = np.linalg.solve(S.toarray(), op.A * phi)
    assert relative_l2(dense[0], lap) < 1e-12


def test_residual_form_start_is_equivalent():
    """Sect. 2.2.2: subtracting S phi from the right-hand side and solving
    for the correction is the same as starting CG from x0 = phi."""
    s = W.icosphere(4, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    op = O.scalar_operator(s, 1)
    phi = O.to_dofs(op, W.sphere_k3_field(s, 1000, n_waves=256))
    k = W.log_scales(s.h, 3)[0]
    S = O.system_matrix(op, k)
    b = op.A * phi
    x1, _, _ = O.pcg_jacobi(S, b, phi, rtol=1e-15)
    d, _, _ = O.pcg_jacobi(S, b - S @ phi, np.zeros_like(phi), rtol=1e-15)
    x0, _, _ = O.pcg_jacobi(S, b, np.zeros_like(phi), rtol=1e-15)
    assert relative_l2(x1, phi + d) < 1e-13
    assert relative_l2(x1, x0) < 1e-13
    assert residual_bound(S, op.A, b, x1) < 1e-13


@pytest.mark.parametrize("n", [1, 2])
def test_filter_invariants_masked_sphere(n):
    s = W.icosphere(4, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    op = O.scalar_operator(s, n)
    phi = W.sphere_k3_field(s, 1001, n_waves=256)
    ks = W.log_scales(s.h, 4)
    out = O.filter_scalar(op, phi, ks)
    pd = O.to_dofs(op, phi)
    # constant in -> constant out (K 1 = 0)
    c = np.where(s.wet.astype(bool), 3.7, 0.0)
    cst = O.filter_scalar(op, c, ks[:2])
    for j in range(2):
        # K_n 1 vanishes up to rounding; S^-1 <= 1/min(A) bounds what that
        # rounding can do to the constant: ||u - 3.7|| <= 3.7 c ||K_n 1|| / min A
        cfac = 0.5 / ks[j] ** (2 * n)
        bound = 3.7 * cfac * np.linalg.norm(op.Kn @ np.ones(op.A.size)) / op.A.min()
        err = np.linalg.norm(O.to_dofs(op, cst[j]) - 3.7)
        assert err <= max(1e-13, 10 * bound), (err, bound)
        assert np.max(np.abs(O.to_dofs(op, cst[j]) - 3.7)) <= 1e-11 * 3.7
    prev = None
    for j in range(len(ks)):
        u = O.to_dofs(op, out[j])
        # area-weighted mean conserved: 1^T K = 0
        assert abs(op.A @ u - op.A @ pd) < 1e-12 * (op.A @ np.abs(pd))
        # M-norm contraction, and monotone in k (eigenvalues 1/(1+c lam))
        eu = op.A @ (u * u)
        assert eu <= op.A @ (pd * pd) * (1 + 1e-14)
        if prev is not None:
            assert eu >= prev * (1 - 1e-14)
        prev = eu
        # dry vertices are returned as zero
        assert np.all(out[j][s.wet == 0] == 0.0)


def test_filter_limits():
    """k -> infinity: the filter is the identity; k -> 0: it returns the
    area-weighted mean (on a connected mesh)."""
    m = W.split_square(32, jitter=0.2)
    op = O.scalar_operator(m, 1)
    phi = W.planar_k3_field(m, 1002)
    hi = O.filter_scalar(op, phi, [1e6])[0]
    assert relative_l2(hi, phi) < 1e-11
    lo = O.filter_scalar(op, phi, [1e-5])[0]
    mean = (op.A @ phi) / op.A.sum()
    assert np.max(np.abs(lo - mean)) < 1e-6 * np.max(np.abs(phi))


def test_cg_certificate_larger_mesh():
    """On a mesh too large for Cholesky the CG + extended-precision
    refinement result carries a certified error bound below 1e-11 (the
    bound itself cannot go below about cond(S) * eps, since storing x in
    FP64 already leaves a residual of ||S|| eps ||x||)."""
    s = W.icosphere(5, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    op = O.scalar_operator(s, 2)
    phi = W.sphere_k3_field(s, 1003, n_waves=256)
    k = W.log_scales(s.h, 5)[0]
    S = O.system_matrix(op, k)
    pd = O.to_dofs(op, phi)
    x, it = O.refine_solve(S, op.A * pd, pd)
    assert residual_bound(S, op.A, op.A * pd, x) < 1e-11
    assert it > 10


def _bound_pins(bound, S, A, b, xs, lam_max):
    """The properties a certificate of ||x - x*|| / ||x|| must have, checked
    around the exact solution xs of S x = b (S = M + c K_n, K_n PSD with
    K_n 1 = 0). Returns the list of failed checks (empty = all hold).

    * x = xs: the bound is at the level of rounding (~ eps cond(S)), at
      least 1000 times below the perturbations used next (1e-6 relative);
    * x = xs + eps 1 (S 1 = M 1, the direction the bound is tight for): it
      bounds the true error and is within RMS(A) / min(A) of it;
    * x = xs + random delta: it bounds the true error and is within
      lam_max(S) / min(A) of it."""
    failed = []
    if not bound(S, A, b, xs) <= 1e-9:
        failed.append("exact solution")
    n = xs.size
    eps = 1e-6 * np.linalg.norm(xs) / np.sqrt(n)
    rng = np.random.default_rng(11)
    for name, d, factor in (
        ("constant", np.full(n, eps), np.sqrt(np.mean(A * A)) / A.min()),
        ("random", eps * rng.standard_normal(n), lam_max / A.min()),
    ):
        x = xs + d
        true = np.linalg.norm(d) / np.linalg.norm(x)
        got = bound(S, A, b, x)
        if not (got >= true * (1 - 1e-6) and got <= factor * true * (1 + 1e-6)):
            failed.append(name)
    return failed


def _mutant_max_area(S, A, b, x):
    """residual_bound with max(A) where min(A) belongs (a planted mistake)."""
    return residual_bound(S, np.full_like(A, A.max()), b, x)


def _mutant_no_mass(S, A, b, x):
    """residual_bound on c K_n alone, the mass term dropped (a planted mistake)."""
    import scipy.sparse as sp

    return residual_bound((S - sp.diags(A)).tocsr(), A, b, x)


@pytest.mark.parametrize("case", ["c1", "sphere5_n2_32h"])
def test_residual_bound_certifies_known_errors(case):
    """The certificate that the full-size GPU tests rely on
    (||x - x*|| / ||x|| <= ||b - S x|| / (min(A) ||x||), since S >= M) checked
    against perturbations of known size around a direct solution: C1, and
    the ill-conditioned biharmonic case (masked level-5 sphere, n = 2, 32h,
    cond(S) ~ 1e5). The same checks reject the oracle with a planted mistake
    (max(A) in place of min(A), or the mass term dropped from the residual)."""
    import scipy.sparse.linalg as spla

    if case == "c1":
        m = W.split_square(64, jitter=0.2)
        op = O.scalar_operator(m, 1)
        phi = W.planar_k3_field(m, 1000)
        k = W.log_scales(1.0, 8)[0]
        method = "dense"
    else:
        m = W.icosphere(5, jitter=0.1)
        m = m.with_mask(W.land_mask(m, 0.3))
        op = O.scalar_operator(m, 2)
        phi = W.sphere_k3_field(m, 1003, n_waves=256)
        k = W.log_scales(m.h, 5)[0]
        method = "direct"
    S = O.system_matrix(op, k)
    pd = O.to_dofs(op, phi)
    b = op.A * pd
    xs = O.filter_scalar(op, phi, [k], method=method)[0]
    xs = O.to_dofs(op, xs)
    lam_max = float(spla.eigsh(S, k=1, which="LA", return_eigenvectors=False)[0]) * 1.001
    assert _bound_pins(residual_bound, S, op.A, b, xs, lam_max) == []
    assert "constant" in _bound_pins(_mutant_max_area, S, op.A, b, xs, lam_max)
    assert "exact solution" in _bound_pins(_mutant_no_mass, S, op.A, b, xs, lam_max)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_shifted_solve_closed_form_all_scales(n):
    """The order-n filter as a sum of order-1 systems with complex shifts
    (S^-1 = (1/n) sum_j (M + s_j b K)^-1, b = c^(1/n)) against the exact
    Fourier multiplier 1 / (1 + gamma (lambda / k^2)^n) on the uniform
    periodic split square, at every scale from 32 to 2 cells, including
    those where S_n itself is too ill-conditioned for a direct solve
    (n = 4 at 32 cells: cond ~1e9)."""
    N = 32
    m = W.split_square(N, jitter=0.0)
    op = O.scalar_operator(m, n)
    phi = W.planar_k3_field(m, 1000)
    ks = W.log_scales(1.0, 5)
    out = O.filter_scalar(op, phi, ks, method="shifted")
    for j, k in enumerate(ks):
        ref = _fourier_filter(phi.reshape(N, N), k, 0.5, n).ravel()
        assert relative_l2(out[j], ref) < 1e-13, (n, j, relative_l2(out[j], ref))


def test_partial_fraction_shifts_identity():
    """(1/n) sum_j 1 / (1 + s_j y) = 1 / (1 + y^n) for y >= 0, n = 1..6 (to
    rounding of the terms, which are O(1 / y) each while the sum is
    O(1 / y^n)), and the shifts come in conjugate pairs (plus s = 1 for odd
    n); no shift lies on the negative real axis, so 1 + s_j y never
    vanishes for y >= 0."""
    y = np.concatenate([[0.0], np.logspace(-3, 3, 61)])
    for n in range(1, 7):
        s = O.solve.partial_fraction_shifts(n)
        lhs = np.mean(1.0 / (1.0 + np.outer(y, s)), axis=1)
        assert np.max(np.abs(lhs.imag)) < 1e-14
        assert np.max(np.abs(lhs.real - 1.0 / (1.0 + y ** n))) < 1e-14
        small = y <= 2.0
        assert np.max(np.abs(lhs.real[small] * (1.0 + y[small] ** n) - 1.0)) < 1e-13
        for sj in s:
            assert np.min(np.abs(s - np.conj(sj))) < 1e-14
            assert not (abs(sj.imag) < 1e-14 and sj.real < 0)
        assert (n % 2 == 1) == bool(np.any(np.abs(s - 1.0) < 1e-14))


@pytest.mark.parametrize("n", [2, 3])
def test_shifted_solve_matches_direct_on_sphere(n):
    """On a jittered, land-masked sphere (no closed form) the shifted route
    equals the direct solve of S_n where S_n is well conditioned (8h .. 2h),
    for scalar vertices and for the vertex vector Laplacian."""
    s = W.icosphere(4, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    phi = W.sphere_k3_field(s, 1000, n_waves=128)
    ks = W.log_scales(s.h, 3, lam_max_cells=8.0)
    op = O.scalar_operator(s, n)
    a = O.filter_scalar(op, phi, ks, method="shifted")
    b = O.filter_scalar(op, phi, ks, method="dense")
    for j in range(len(ks)):
        assert relative_l2(a[j], b[j]) < 1e-12, (j, relative_l2(a[j], b[j]))
    wet = np.array(W.land_mask(s, 0.3), dtype=np.uint8)
    wet[np.abs(s.coords[:, 2] / s.radius) > np.sin(np.radians(80))] = 0
    sv = s.with_mask(wet)
    opv = O.vertex_vector_operator(sv, n)
    u = W.sphere_k3_velocity(sv, 31, 32, n_waves=64)
    rhs = O.project_cells_to_vertices(opv, u)
    for k in ks:
        x1 = O.solve.shifted_solve(opv, rhs, float(k))
        x2 = O.solve.filter_dense(O.system_matrix(opv, float(k)), rhs)
        assert relative_l2(x1, x2) < 1e-12
