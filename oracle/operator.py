"""Frozen SIMP operator, direct solve and relative residual.

* Ersatz SIMP law, Eq. (floor_scaling): E_e = rho_min + (1 - rho_min) rho_e^p.
  Stored densities are floor-independent (Sec. 3.2); a voxel "at the floor" is
  stored as rho = 0 so that E_e = rho_min exactly.
* Frozen operator, Eq. (frozen_operator): K(rho_min) = sum_e E_e K_e restricted
  to the free DOFs.
* Relative residual, Eq. (relative_residual): eta = ||f - K u|| / ||f|| over the
  free DOFs, in FP64 (Tab. residual-semantics, "recomputed true residual").
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .ke import LOCAL


def young(rho, p, rho_min):
    """Eq. (floor_scaling).  rho must lie in [0, 1]."""
    rho = np.asarray(rho, dtype=float)
    if not np.all(np.isfinite(rho)) or rho.min(initial=0.0) < 0 or rho.max(initial=0.0) > 1:
        raise ValueError("densities must be finite and in [0, 1]")
    if not (0 < rho_min <= 1) or not (p > 0):
        raise ValueError("need 0 < rho_min <= 1 and p > 0")
    return rho_min + (1.0 - rho_min) * rho ** p


def assemble(grid, E, Ke):
    """Full (unconstrained) n_dof x n_dof CSR matrix sum_e E_e A_e^T Ke A_e."""
    dofs = grid.elem_dofs()
    rows = np.repeat(dofs, 24, axis=1).ravel()
    cols = np.tile(dofs, (1, 24)).ravel()
    vals = (np.asarray(E)[:, None] * Ke.ravel()[None, :]).ravel()
    K = sp.coo_matrix((vals, (rows, cols)), shape=(grid.n_dof, grid.n_dof)).tocsr()
    K.sum_duplicates()
    return K


def free_block(K, free):
    idx = np.flatnonzero(free)
    return K[idx][:, idx].tocsc()


def apply_full(grid, E, Ke, u, chunk=1 << 18):
    """y = K u by element loops (matrix-free, for grids too large to assemble).

    u is a full-length vector; constrained entries of u are treated as zero and
    constrained entries of y are set to zero (the free-DOF operator)."""
    free = grid.free_dofs()
    u = np.where(free, u, 0.0)
    y = np.zeros(grid.n_dof)
    dofs = grid.elem_dofs()
    E = np.asarray(E)
    for s in range(0, grid.n_elem, chunk):
        d = dofs[s:s + chunk]
        ue = u[d]                                   # (c, 24)
        ve = (ue @ Ke.T) * E[s:s + chunk, None]     # Ke symmetric
        np.add.at(y, d.ravel(), ve.ravel())
    y[~free] = 0.0
    return y


def apply_at_node(grid, E, Ke, u, n):
    """The three entries of K u at node n, from the element definition alone
    (used for sampled checks at sizes the assembled oracle cannot hold)."""
    i, j, k = grid.node_ijk(n)
    out = np.zeros(3)
    if i == 0:
        return out
    for a, (di, dj, dk) in enumerate(LOCAL):
        ex, ey, ez = i - di, j - dj, k - dk
        if not (0 <= ex < grid.nx and 0 <= ey < grid.ny and 0 <= ez < grid.nz):
            continue
        e = ex + grid.nx * (ey + grid.ny * ez)
        ue = np.zeros(24)
        for b, (bi, bj, bk) in enumerate(LOCAL):
            if ex + bi == 0:             # clamped node (x = 0 face): zero DOFs
                continue
            m = grid.node(ex + bi, ey + bj, ez + bk)
            ue[3 * b:3 * b + 3] = u[3 * m:3 * m + 3]
        out += E[e] * (Ke[3 * a:3 * a + 3, :] @ ue)
    return out


def solve_direct(K_ff, f_f):
    """u* = K_ff^{-1} f_f by sparse LU (SuperLU), FP64."""
    return spla.splu(sp.csc_matrix(K_ff)).solve(f_f)


def _ratio(nr, nf):
    """||r|| / ||f||.  Eq. (relative_residual) is undefined for f = 0; the
    reading taken: 0 when r = 0 as well (u = 0 solves f = 0 exactly), NaN for
    every other case where ||f|| is not a finite positive number."""
    if nr == 0.0 and nf == 0.0:
        return 0.0
    if not (nf > 0.0 and np.isfinite(nf)):
        return float("nan")
    return float(nr / nf)


def relative_residual(K_ff, f_f, u_f):
    """Eq. (relative_residual) on free DOFs."""
    return _ratio(np.linalg.norm(f_f - K_ff @ u_f), np.linalg.norm(f_f))


def relative_residual_full(grid, E, Ke, f, u):
    """Eq. (relative_residual) with the matrix-free operator, for grids too
    large to assemble: f, u are full-length vectors, norms over free DOFs."""
    free = grid.free_dofs()
    r = np.where(free, f, 0.0) - apply_full(grid, E, Ke, u)
    return _ratio(np.linalg.norm(r[free]), np.linalg.norm(f[free]))


def residual_bound(K_ff, f_f, u_f):
    """A rounding bound for evaluating eta in FP64: n_row_nnz * eps *
    || |K||u| + |f| || / ||f||.  Used to flag boundary-ambiguous accepts."""
    absK = abs(K_ff)
    nnz_row = int(np.diff(sp.csr_matrix(K_ff).indptr).max())
    eps = np.finfo(float).eps
    return float(nnz_row * eps * np.linalg.norm(absK @ np.abs(u_f) + np.abs(f_f)) / np.linalg.norm(f_f))


def residual_bound_full(grid, E, Ke, f, u):
    """The bound of residual_bound without assembling K: |K| |u| <= sum_e E_e
    |K_e| |u_e| entrywise (E_e > 0), and a free row of the hex8 operator has
    at most 81 nonzeros (27 nodes x 3 components)."""
    free = grid.free_dofs()
    a = apply_full(grid, E, np.abs(Ke), np.abs(u))
    eps = np.finfo(float).eps
    return float(81 * eps * np.linalg.norm((a + np.abs(f))[free]) / np.linalg.norm(f[free]))


def compliance(f_f, u_f):
    return float(f_f @ u_f)
