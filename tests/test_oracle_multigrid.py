"""Pins of the oracle's V-cycle (Tab. solver-config: 2:1 trilinear transfer,
Galerkin coarse operators; fixed linear V-cycle with damped node-block Jacobi)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ke, mesh
from oracle import multigrid as mg
from oracle import operator as op

Ke = ke.ke()


@pytest.mark.parametrize("dims,levels,coarsest", [
    ((16, 8, 8), 3, (4, 2, 2)), ((64, 32, 32), 5, (4, 2, 2)), ((32, 16, 16), 4, (4, 2, 2)),
    ((48, 24, 24), 4, (6, 3, 3)), ((96, 48, 48), 5, (6, 3, 3)), ((256, 128, 128), 7, (4, 2, 2))])
def test_level_rule(dims, levels, coarsest):
    d = mg.level_dims(*dims)
    assert len(d) == levels and d[-1] == coarsest


def test_prolongation_interpolates_linear_fields():
    fg_, cg = mesh.Grid(8, 4, 6), mesh.Grid(4, 2, 3)
    P = mg.prolongation(fg_, cg)
    rng = np.random.default_rng(0)
    A, t = rng.standard_normal((3, 3)), rng.standard_normal(3)
    uc = (cg.node_coords() * 2 @ A.T + t).ravel()      # coarse node spacing is 2
    uf = (fg_.node_coords() @ A.T + t).ravel()
    assert np.max(np.abs(P @ uc - uf)) < 1e-13
    assert set(np.round(P.data, 12)) <= {1.0, 0.5, 0.25, 0.125}


def test_galerkin_uniform_equals_rediscretized():
    # nested FE spaces: P^T K_h P is the coarse-space stiffness; a cubic element
    # of edge 2 has stiffness 2 * Ke (3D elasticity scales with h)
    fgd, cgd = mesh.Grid(8, 4, 4), mesh.Grid(4, 2, 2)
    H = mg.build_hierarchy(fgd, np.full(fgd.n_elem, 0.3), Ke)
    Kc = op.free_block(op.assemble(cgd, np.full(cgd.n_elem, 0.3 * 2.0), Ke), cgd.free_dofs())
    assert abs(H[1].K - Kc).max() < 1e-14


def test_node_block_inverse_and_smoother_bound():
    g = mesh.Grid(16, 8, 8)
    E = op.young(np.random.default_rng(0).random(g.n_elem), 3, 1e-3)
    H = mg.build_hierarchy(g, E, Ke)
    K = H[0].K.toarray()
    Binv = H[0].Binv.toarray()
    for b in range(0, 30, 3):
        assert np.allclose(Binv[b:b + 3, b:b + 3] @ K[b:b + 3, b:b + 3], np.eye(3), atol=1e-12)
    # damped node-block Jacobi with w = 0.6 is a convergent smoother: w * lmax < 2
    lmax = sp.linalg.eigsh(sp.csr_matrix(H[0].Binv @ H[0].K), k=1, which="LM",
                           return_eigenvectors=False)[0]
    assert 0.6 * lmax < 2.0


def test_single_level_is_direct_solve():
    g = mesh.Grid(4, 2, 2)
    E = op.young(np.random.default_rng(1).random(g.n_elem), 3, 1e-3)
    H = mg.build_hierarchy(g, E, Ke, max_levels=1)
    b = np.random.default_rng(2).standard_normal(H[0].K.shape[0])
    x = mg.vcycle(H, b)
    assert np.linalg.norm(H[0].K @ x - b) < 1e-12 * np.linalg.norm(b)


def _closed_form_minv(H, omega=0.6, nu1=2, nu2=2, l=0):
    """M_l^-1 = (I - S^nu2 (I - P M_{l+1}^-1 P^T K) S^nu1) K^-1 with
    S = I - w B^-1 K (error-propagation form, dense)."""
    L = H[l]
    K = L.K.toarray()
    n = K.shape[0]
    Kinv = np.linalg.inv(K)
    if L.P is None:
        return Kinv
    S = np.eye(n) - omega * L.Binv.toarray() @ K
    P = L.P.toarray()
    C = np.eye(n) - P @ _closed_form_minv(H, omega, nu1, nu2, l + 1) @ P.T @ K
    Eprop = np.linalg.matrix_power(S, nu2) @ C @ np.linalg.matrix_power(S, nu1)
    return (np.eye(n) - Eprop) @ Kinv


@pytest.mark.parametrize("dims,rmin,nlev", [((8, 4, 4), 1e-3, 2), ((8, 8, 8), 1.0, 3),
                                           ((8, 8, 8), 1e-3, 3)])
def test_vcycle_matches_error_propagation_form(dims, rmin, nlev):
    g = mesh.Grid(*dims)
    E = op.young(np.random.default_rng(3).random(g.n_elem), 3, rmin)
    H = mg.build_hierarchy(g, E, Ke, max_coarse_dof=100)
    assert len(H) == nlev
    M = mg.vcycle_matrix(H)
    Mc = _closed_form_minv(H)
    assert np.max(np.abs(M - Mc)) <= 1e-9 * np.max(np.abs(M))
    # fixed symmetric smoothing pre and post: M^-1 symmetric positive definite
    assert np.max(np.abs(M - M.T)) <= 1e-11 * np.max(np.abs(M))
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    # error contraction of the V-cycle is below 1
    K = H[0].K.toarray()
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(K.shape[0]) - M @ K)))
    assert rho < 1.0


def test_free_dof_count_equals_the_grid_mask():
    from oracle import mesh
    for dims in ((1, 1, 1), (4, 2, 2), (16, 8, 8), (17, 9, 7), (64, 32, 32)):
        assert mg.free_dof_count(*dims) == int(mesh.Grid(*dims).free_dofs().sum())
