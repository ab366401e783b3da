"""The filter solve (oracle, FP64, test-only).

Eq. 1 with the discrete operators of Sect. 2.1.1 (Eq. 4 / Eq. 5 forms):
``S = M + gamma * k^(-2n) * K_n``, ``S phi_bar = M phi``, with ``k = 1/l``
and ``gamma = 1/2`` (Sect. 2.1). ``S`` is symmetric positive definite
(Sect. 2.1.1), so ``phi_bar = S^-1 M phi`` is unique; the oracle computes it

* by dense Cholesky for small systems,
* (``method="shifted"``, orders n >= 2) as a sum of order-1 systems with
  complex shifts, each by sparse LU (``shifted_solve``), and
* by Jacobi-preconditioned conjugate gradients started from ``x0 = phi``
  (the residual form of Sect. 2.2.2: the product ``S phi`` is subtracted
  from the right-hand side and CG solves for the correction), to a tight
  tolerance, followed by iterative refinement whose residual is formed in
  extended (x87 80-bit) precision.
"""
from __future__ import annotations


import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def system_matrix(op, k: float, gamma: float = 0.5):
    """``S = M + c K_n`` with ``c = gamma / k^(2n)`` (Eq. 1, Eq. 4/5)."""
    c = gamma / (k ** (2 * op.n))
    return (sp.diags(op.A) + c * op.Kn).tocsr()


def _cell_scalar(op) -> bool:
    return op.A.size == op.cells.size if hasattr(op, "cells") else False


def to_dofs(op, field: np.ndarray) -> np.ndarray:
    """Caller's numbering (vertices or cells) -> dof vector."""
    if hasattr(op, "verts"):
        return np.asarray(field, dtype=np.float64)[op.verts]
    if _cell_scalar(op):
        return np.asarray(field, dtype=np.float64)[op.cells]
    f = np.asarray(field, dtype=np.float64).reshape(-1, 2)
    return f[op.cells].reshape(-1)


def from_dofs(op, x: np.ndarray) -> np.ndarray:
    """dof vector -> caller's numbering, zeros at dry vertices / cells."""
    if hasattr(op, "verts"):
        out = np.zeros(op.n_vertices)
        out[op.verts] = x
        return out
    if _cell_scalar(op):
        out = np.zeros(op.n_cells_total)
        out[op.cells] = x
        return out
    out = np.zeros((op.n_cells_total, 2))
    out[op.cells] = x.reshape(-1, 2)
    return out.reshape(-1)


def filter_dense(S, b) -> np.ndarray:
    """Dense Cholesky solve of the SPD system (small meshes only)."""
    Sd = S.toarray() if sp.issparse(S) else np.asarray(S)
    cf = sla.cho_factor(Sd, lower=True)
    return sla.cho_solve(cf, b)


def pcg_jacobi(S, b, x0, rtol: float = 1e-14, max_iter: int = 100000, replace_every: int = 50):
    """Jacobi-preconditioned CG on ``S x = b`` from ``x0``, FP64.

    Stops when the true residual satisfies ``||b - S x|| <= rtol ||b||``
    (the recursive residual is replaced by the true one every
    ``replace_every`` iterations) or when it stops decreasing.
    Returns ``(x, iterations, true_relative_residual)``.
    """
    S = S.tocsr()
    d = S.diagonal()
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - S @ x
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(x), 0, 0.0
    z = r / d
    p = z.copy()
    rho = float(r @ z)
    best = np.linalg.norm(r)
    stall = 0
    it = 0
    while it < max_iter:
        if np.linalg.norm(r) <= rtol * bn:
            break
        q = S @ p
        alpha = rho / float(p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        if it % replace_every == 0:
            r = b - S @ x
            rn = np.linalg.norm(r)
            if rn < 0.5 * best:
                best = rn
                stall = 0
            else:
                stall += 1
                if stall >= 3:
                    break
        z = r / d
        rho_new = float(r @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    res = np.linalg.norm(b - S @ x) / bn
    return x, it, res


def refine_solve(S, b, x0, steps: int = 3, rtol: float = 1e-14):
    """CG from ``x0`` followed by ``steps`` rounds of iterative refinement
    with an extended-precision residual. Returns ``(x, total_iterations)``."""
    x, it, _ = pcg_jacobi(S, b, x0, rtol=rtol)
    xl = x.astype(np.longdouble)
    bn = float(np.linalg.norm(b))
    for _ in range(steps):
        r = _residual_ld(S, b, xl)
        r64 = r.astype(np.float64)
        rn = float(np.linalg.norm(r64))
        if rn <= 1e-17 * bn:
            break
        d, it2, _ = pcg_jacobi(S, r64, np.zeros_like(r64), rtol=rtol)
        it += it2
        xl = xl + d.astype(np.longdouble)
    return xl.astype(np.float64), it


def _residual_ld(S, b, xl):
    """``b - S x`` with products and sums in x87 extended precision
    (``xl`` is already extended)."""
    ld = np.longdouble
    prod = S.data.astype(ld) * xl[S.indices]
    nnz_row = np.diff(S.indptr)
    sx = np.zeros(S.shape[0], dtype=ld)
    nz = nnz_row > 0
    sx[nz] = np.add.reduceat(prod, S.indptr[:-1][nz])
    return b.astype(ld) - sx


def direct_refine_solve(S, b, steps: int = 3):
    """Sparse LU of ``S`` (a library factorisation) followed by ``steps``
    rounds of iterative refinement with an extended-precision residual; for
    the ill-conditioned systems of n = 2 at large scales, where CG
    stagnates long before the plain definition S^-1 M phi is reached (the
    convergence loss the paper reports for the biharmonic filter at large
    scales, Sect. 6)."""
    lu = spla.splu(S.tocsc())
    xl = lu.solve(b).astype(np.longdouble)
    bn = float(np.linalg.norm(b))
    for _ in range(steps):
        r = _residual_ld(S, b, xl)
        r64 = r.astype(np.float64)
        if float(np.linalg.norm(r64)) <= 1e-17 * bn:
            break
        xl = xl + lu.solve(r64).astype(np.longdouble)
    return xl.astype(np.float64)


def partial_fraction_shifts(n: int) -> np.ndarray:
    """Shifts ``s_j`` of ``1 / (1 + y^n) = (1/n) sum_j 1 / (1 + s_j y)``:
    ``s_j = -1 / w_j`` over the ``n`` roots ``w_j = exp(i pi (2j + 1) / n)``
    of ``w^n = -1`` (the residue of ``1 / (1 + y^n)`` at ``w`` is
    ``1 / (n w^(n-1)) = -w / n``). Conjugate roots give conjugate shifts."""
    w = np.exp(1j * np.pi * (2 * np.arange(n) + 1) / n)
    return -1.0 / w


def shifted_solve(op, b, k: float, gamma: float = 0.5) -> np.ndarray:
    """``S^-1 b`` for ``S = M + c K_n`` through order-1 systems only.

    ``K_n = K (M^-1 K)^(n-1)`` gives ``S = M (I + c T^n)`` with ``T = M^-1 K``,
    whose eigenvalues are real and nonnegative (``K`` symmetric positive
    semidefinite, ``M`` diagonal positive). The scalar identity of
    ``partial_fraction_shifts`` with ``y = b x``, ``b = c^(1/n)``, applied to
    ``T`` gives ``S^-1 = (1/n) sum_j (M + s_j b K)^-1``. Every shifted matrix
    is solved by complex sparse LU (a library factorisation); the shifts
    come in conjugate pairs (and ``s = 1`` for odd n), so the sum is real.
    The shifted systems are well conditioned (``|1 + s_j b x| >= sin(pi/n)``
    for ``n >= 2``), which keeps this route accurate where ``S`` itself is
    not (n >= 3 at large scales)."""
    n = op.n
    c = gamma / (k ** (2 * n))
    bn = c ** (1.0 / n)
    M = sp.diags(op.A)
    K = op.K.tocsr()
    out = np.zeros(b.size)
    for s in partial_fraction_shifts(n):
        if s.imag < -1e-12:
            continue  # the conjugate of a shift already solved
        if abs(s.imag) <= 1e-12:
            A = (M + (s.real * bn) * K).tocsc()
            out += spla.splu(A).solve(b) / n
        else:
            A = (M.astype(np.complex128) + (s * bn) * K).tocsc()
            out += 2.0 * spla.splu(A).solve(b.astype(np.complex128)).real / n
    return out


def _solve(op, phi_dofs, k, gamma, method):
    return _solve_rhs(op, op.A * phi_dofs, phi_dofs, k, gamma, method)


def _solve_rhs(op, b, x0, k, gamma, method):
    """Solve ``S x = b``; ``x0`` starts the iterative method."""
    S = system_matrix(op, k, gamma)
    phi_dofs = x0
    n = b.size
    if method == "auto":
        method = "dense" if n <= 4096 else ("direct" if n <= 300_000 else "cg")
    if method == "dense":
        return filter_dense(S, b), {"method": "dense", "iterations": 0}
    if method == "direct":
        return direct_refine_solve(S, b), {"method": "direct", "iterations": 0}
    if method == "shifted":
        return shifted_solve(op, b, k, gamma), {"method": "shifted", "iterations": 0}
    x, it = refine_solve(S, b, phi_dofs)
    return x, {"method": "cg", "iterations": it}


def filter_scalar(op, field, ks, gamma: float = 0.5, method: str = "auto", return_info: bool = False):
    """Filter a scalar field at each wavenumber in ``ks``.

    ``field``: (V,) in vertex numbering (vertex placements) or (F,) in
    triangle numbering (circumcentre placement). Returns (len(ks), V or F)
    with zeros at entries that are not dofs (dry, orphaned, inactive).
    """
    phi = to_dofs(op, field)
    out = np.zeros((len(ks), op.n_vertices if hasattr(op, "verts") else op.n_cells_total))
    infos = []
    for j, k in enumerate(ks):
        x, info = _solve(op, phi, float(k), gamma, method)
        out[j] = from_dofs(op, x)
        infos.append(info)
    return (out, infos) if return_info else out


def filter_vector(op, field, ks, gamma: float = 0.5, method: str = "auto", return_info: bool = False):
    """Filter a cell vector field ``(F, 2)`` (east, north) at each ``k``.
    Returns (len(ks), F, 2) with zeros on inactive cells."""
    phi = to_dofs(op, field)
    out = np.zeros((len(ks), op.n_cells_total, 2))
    infos = []
    for j, k in enumerate(ks):
        x, info = _solve(op, phi, float(k), gamma, method)
        out[j] = from_dofs(op, x).reshape(-1, 2)
        infos.append(info)
    return (out, infos) if return_info else out


def project_cells_to_vertices(op, cell_field) -> np.ndarray:
    """Right-hand side of the vertex vector filter (Sect. 2.1.2):
    ``R_vc u_c`` over active cells, interleaved ``(east, north)`` per dof.
    ``cell_field``: (F, 2) in triangle numbering."""
    u = np.asarray(cell_field, dtype=np.float64).reshape(-1)
    return op.Rvc @ u


def filter_vertex_vector(op, cell_field, ks, gamma: float = 0.5, method: str = "auto",
                         return_info: bool = False):
    """Filter a cell velocity field ``(F, 2)`` onto vertices at each ``k``:
    ``S x = R_vc u_c`` with ``S = M_2 + gamma/k^(2n) K_n`` (Sect. 2.1.2).
    Returns (len(ks), V, 2) (east, north) with zeros at vertices that are
    not dofs; the iterative method starts from ``M_2^-1 R_vc u_c``."""
    b = project_cells_to_vertices(op, cell_field)
    x0 = b / op.A
    out = np.zeros((len(ks), op.n_vertices, 2))
    infos = []
    for j, k in enumerate(ks):
        x, info = _solve_rhs(op, b, x0, float(k), gamma, method)
        out[j][op.verts] = x.reshape(-1, 2)
        infos.append(info)
    return (out, infos) if return_info else out


def residual_bound(S, A, b, x) -> float:
    """Certified bound on the relative error of ``x``: since ``K_n`` is
    positive semidefinite, ``S >= M`` and ``||S^-1|| <= 1/min(A)``, so
    ``||x - x*|| / ||x|| <= ||b - S x|| / (min(A) ||x||)``; the residual is
    formed in extended precision so that its own rounding does not hide
    the bound."""
    r = _residual_ld(S.tocsr(), np.asarray(b, dtype=np.float64), np.asarray(x).astype(np.longdouble))
    return float(np.linalg.norm(r.astype(np.float64)) / (np.min(A) * np.linalg.norm(x)))


def relative_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


__all__ = [
    "system_matrix",
    "to_dofs",
    "from_dofs",
    "filter_dense",
    "pcg_jacobi",
    "refine_solve",
    "filter_scalar",
    "filter_vector",
    "residual_bound",
    "relative_l2",
]
