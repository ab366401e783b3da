"""The iteration form of the batched engine, in plain NumPy, against textbook PCG.

The batched kernels run Jacobi-preconditioned CG (COCG for the complex-shifted
order-2 solves) in chunks of four iterations without a direction vector:

  * chunk start: z_0 = r / d from the FP64 true residual r = b - S x, rho =
    (r, z_0), beta_0 = rho / rho_prev (0 for a new column);
  * iteration 0: p_0 = z_0 + beta_0 p_-1, u_0 = d^-1 S p_0, (p_0, q_0) summed
    directly (q = S p = d u);
  * iteration k >= 1: z_k = z_k-1 - alpha_k-1 u_k-1, u_k = d^-1 S z_k +
    beta_k u_k-1, and (p_k, q_k) = (z_k, q_k) + beta_k ((q_k-1, z_k) +
    beta_k (p_k-1, q_k-1)), which holds for any S with S^T = S;
  * alpha_k = rho_k / (p_k, q_k), and the next rho from rho - 2 alpha (q, z) +
    alpha^2 (q, d^-1 q), so beta_k+1 is known before z_k+1 exists;
  * chunk end: p_k = z_k + beta_k p_k-1 rebuilt from the stored z_k and the
    carried p_-1, x += sum_k alpha_k p_k, p_3 carried to the next chunk.

In exact arithmetic every chunk reproduces four iterations of textbook PCG
(and the replacement residual equals the recursive one), so in FP64 the
iterates agree to rounding. These tests pin that algebra, independent of the
HIP kernels and of the oracle's own solver.
"""
import numpy as np
import scipy.sparse as sp

L = 4  # iterations per chunk


def grid_laplacian(nx, ny, seed):
    """Weighted 5-point graph Laplacian on an nx x ny grid (random positive
    edge weights): symmetric, positive semidefinite."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    idx = np.arange(n).reshape(nx, ny)
    rows, cols, vals = [], [], []
    for a, b in ((idx[:-1, :], idx[1:, :]), (idx[:, :-1], idx[:, 1:])):
        w = rng.uniform(0.5, 1.5, a.size)
        for i, j in ((a.ravel(), b.ravel()), (b.ravel(), a.ravel())):
            rows.append(i)
            cols.append(j)
            vals.append(-w)
    k_off = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return k_off - sp.diags(np.asarray(k_off.sum(axis=1)).ravel())


def textbook_pcg(S, b, x0, d, iters):
    """Jacobi-PCG as printed in any textbook (real or complex-symmetric:
    the inner product is the bilinear x^T y)."""
    x = x0.copy()
    r = b - S @ x
    z = r / d
    p = z.copy()
    rho = r @ z
    for _ in range(iters):
        q = S @ p
        a = rho / (p @ q)
        x = x + a * p
        r = r - a * q
        z = r / d
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x


def chunked_zu(S, b, x0, d, chunks):
    """The batched engine's form (module docstring), in FP64."""
    x = x0.copy()
    p_carry = np.zeros_like(x0)
    rho_prev = None
    for _ in range(chunks):
        r = b - S @ x  # FP64 replacement (at a new column: the start pass)
        z = [r / d]
        rho = r @ z[0]
        beta = 0.0 if rho_prev is None else rho / rho_prev
        alphas, betas = [], []
        u_prev = pq_prev = None
        for k in range(L):
            if k == 0:
                p0 = z[0] + beta * p_carry
                u = (S @ p0) / d
                pq = p0 @ (d * u)
                zk = z[0]
            else:
                zk = z[k - 1] - alphas[-1] * u_prev
                z.append(zk)
                u = (S @ zk) / d + beta * u_prev
                zu, xz = zk @ (d * u), (d * u_prev) @ zk
                pq = zu + beta * (xz + beta * pq_prev)
                rho = zk @ (d * zk)  # the kernel's exact (r, z) of the z it formed
            a = rho / pq
            alphas.append(a)
            betas.append(beta)
            # next rho before the next z exists
            rho_next = rho - 2.0 * a * (zk @ (d * u)) + a * a * ((d * u) @ u)
            beta = rho_next / rho
            u_prev, pq_prev = u, pq
        # the chunk's x update: rebuild the directions from z_0..z_3 and p_-1
        pk = p_carry
        for k in range(L):
            pk = z[k] + betas[k] * pk
            x = x + alphas[k] * pk
        p_carry = pk
        rho_prev = rho
    return x


def test_chunked_form_matches_textbook_pcg_real():
    K = grid_laplacian(24, 20, seed=3)
    n = K.shape[0]
    rng = np.random.default_rng(5)
    mass = rng.uniform(0.5, 2.0, n)
    c = 40.0
    S = (sp.diags(mass) + c * K).tocsr()
    d = S.diagonal()
    phi = rng.standard_normal(n)
    b = mass * phi
    for chunks in (1, 3, 6):
        ref = textbook_pcg(S, b, phi, d, L * chunks)
        got = chunked_zu(S, b, phi, d, chunks)
        sol = sp.linalg.spsolve(S.tocsc(), b)
        err_ref = np.linalg.norm(ref - sol)
        assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(sol), chunks
        # and it is the same iterate, not merely a converged one
        if err_ref > 1e-6 * np.linalg.norm(sol):
            assert np.linalg.norm(got - ref) <= 1e-6 * err_ref, chunks


def test_chunked_form_matches_textbook_cocg_complex_symmetric():
    # the order-2 filter's shifted system M + sigma K, sigma complex: S^T = S,
    # not Hermitian; COCG uses the bilinear form, as the complex tiles do
    K = grid_laplacian(18, 16, seed=7)
    n = K.shape[0]
    rng = np.random.default_rng(9)
    mass = rng.uniform(0.5, 2.0, n)
    sigma = -np.cos(np.pi / 4) * 6.0 + 1j * np.sin(np.pi / 4) * 6.0
    S = (sp.diags(mass.astype(complex)) + sigma * K).tocsr()
    d = S.diagonal()
    phi = rng.standard_normal(n).astype(complex)
    b = mass * phi
    for chunks in (1, 2, 5):
        ref = textbook_pcg(S, b, phi, d, L * chunks)
        got = chunked_zu(S, b, phi, d, chunks)
        sol = sp.linalg.spsolve(S.tocsc(), b)
        err_ref = np.linalg.norm(ref - sol)
        assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(sol), chunks
        if err_ref > 1e-6 * np.linalg.norm(sol):
            assert np.linalg.norm(got - ref) <= 1e-6 * err_ref, chunks


def test_pq_identity_needs_symmetry():
    # the (p, q) identity is where symmetry enters: with a nonsymmetric S the
    # chunked form leaves textbook PCG after the first iteration of a chunk
    K = grid_laplacian(12, 12, seed=11)
    n = K.shape[0]
    rng = np.random.default_rng(13)
    S = (sp.eye(n) * 2.0 + 5.0 * K).tolil()
    S[0, 1] += 0.8  # break S^T = S
    S = S.tocsr()
    d = S.diagonal()
    phi = rng.standard_normal(n)
    b = phi.copy()
    ref = textbook_pcg(S, b, phi, d, L)
    got = chunked_zu(S, b, phi, d, 1)
    assert np.linalg.norm(got - ref) > 1e-8 * np.linalg.norm(ref)
