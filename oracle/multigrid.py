"""Geometric multigrid preconditioner (Tab. solver-config; Sec. 4.5.3).

The paper's hierarchy uses 2:1 trilinear transfers and Galerkin coarse
operators.  The preconditioner built here is the fixed linear V-cycle of the
paper's control configuration (adaptive coarse/fine corrections disabled):

  level l, input b:
    x = w B^-1 b                      (first pre-sweep from zero)
    x = x + w B^-1 (b - K x)          (remaining pre-sweeps)
    r = b - K x;  b_c = P^T r;  e_c = Vcycle(l+1, b_c);  x = x + P e_c
    x = x + w B^-1 (b - K x)          (post-sweeps)
  coarsest level: x = K_L^-1 b by dense Cholesky (FP64 direct coarse solve).

Readings (the paper is silent on these):
* "damped Jacobi" is the 3x3 node-block Jacobi B (one dense block per mesh node
  coupling u_x, u_y, u_z, the node-block operator of Tab. solver-config), w=0.6;
* levels: coarsen 2:1 while all element counts are even, every coarse count stays
  >= 2 and the current level has more than ``max_coarse_dof`` free DOFs;
* coarse boundary conditions: the coarse x = 0 nodes are clamped.  Fine x = 0
  nodes interpolate only from coarse x = 0 nodes, so restricting P to free rows
  and free columns is exact.

All matrices here act on free-DOF vectors.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .mesh import Grid
from .operator import assemble, free_block


def free_dof_count(nx, ny, nz):
    return 3 * nx * (ny + 1) * (nz + 1)


def level_dims(nx, ny, nz, max_coarse_dof=300, max_levels=0):
    dims = [(nx, ny, nz)]
    while True:
        if max_levels and len(dims) >= max_levels:
            break
        x, y, z = dims[-1]
        if free_dof_count(x, y, z) <= max_coarse_dof:
            break
        if x % 2 or y % 2 or z % 2:
            break
        if x // 2 < 2 or y // 2 < 2 or z // 2 < 2:
            break
        dims.append((x // 2, y // 2, z // 2))
    return dims


def _weights_1d(i):
    """Coarse parents of fine index i with trilinear weights."""
    if i % 2 == 0:
        return [(i // 2, 1.0)]
    return [((i - 1) // 2, 0.5), ((i + 1) // 2, 0.5)]


def prolongation(fine, coarse):
    """Full-DOF trilinear prolongation (fine n_dof x coarse n_dof), per component."""
    rows, cols, vals = [], [], []
    for k in range(fine.NZ):
        wk = _weights_1d(k)
        for j in range(fine.NY):
            wj = _weights_1d(j)
            for i in range(fine.NX):
                wi = _weights_1d(i)
                fn = fine.node(i, j, k)
                for (I, a) in wi:
                    for (J, b) in wj:
                        for (K, c) in wk:
                            cn = coarse.node(I, J, K)
                            for comp in range(3):
                                rows.append(3 * fn + comp)
                                cols.append(3 * cn + comp)
                                vals.append(a * b * c)
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.n_dof, coarse.n_dof))


def node_block_inverse(K_ff):
    """Block-diagonal inverse of the 3x3 node blocks of a free-DOF matrix.
    Free DOFs come in whole-node triples, so consecutive triples are blocks."""
    n = K_ff.shape[0]
    Kc = sp.csr_matrix(K_ff)
    blocks = np.zeros((n // 3, 3, 3))
    for r in range(3):
        for c in range(3):
            blocks[:, r, c] = np.asarray(Kc[np.arange(r, n, 3), np.arange(c, n, 3)]).ravel()
    inv = np.linalg.inv(blocks)
    return sp.block_diag(list(inv), format="csr")


class Level:
    pass


def build_hierarchy(grid, E, Ke, max_coarse_dof=300, max_levels=0):
    """Assembled free-DOF hierarchy: K_0 from the element definition, then
    Galerkin K_{l+1} = P_l^T K_l P_l; node-block inverses; coarsest Cholesky."""
    dims = level_dims(grid.nx, grid.ny, grid.nz, max_coarse_dof, max_levels)
    grids = [grid] + [Grid(*d) for d in dims[1:]]
    levels = []
    K = free_block(assemble(grid, E, Ke), grid.free_dofs())
    for l, g in enumerate(grids):
        L = Level()
        L.grid = g
        L.K = sp.csr_matrix(K)
        L.Binv = node_block_inverse(L.K)
        if l + 1 < len(grids):
            cg = grids[l + 1]
            P = prolongation(g, cg)
            ff = np.flatnonzero(g.free_dofs())
            fc = np.flatnonzero(cg.free_dofs())
            L.P = sp.csr_matrix(P[ff][:, fc])
            K = L.P.T @ L.K @ L.P
        else:
            L.P = None
            L.chol = sla.cho_factor(L.K.toarray(), lower=True)
        levels.append(L)
    return levels


def vcycle(levels, b, omega=0.6, nu_pre=2, nu_post=2, l=0):
    """One fixed V-cycle z = M^-1 b on free-DOF vectors."""
    L = levels[l]
    if L.P is None:
        return sla.cho_solve(L.chol, b)
    x = omega * (L.Binv @ b)
    for _ in range(nu_pre - 1):
        x = x + omega * (L.Binv @ (b - L.K @ x))
    r = b - L.K @ x
    ec = vcycle(levels, L.P.T @ r, omega, nu_pre, nu_post, l + 1)
    x = x + L.P @ ec
    for _ in range(nu_post):
        x = x + omega * (L.Binv @ (b - L.K @ x))
    return x


def vcycle_matrix(levels, **kw):
    """Dense M^-1 (small grids only), column by column."""
    n = levels[0].K.shape[0]
    M = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, c] = vcycle(levels, e, **kw)
    return M
