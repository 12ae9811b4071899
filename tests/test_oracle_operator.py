"""Pins of the oracle's grid, SIMP law, assembly and direct solve
(Eqs. floor_scaling, frozen_operator, relative_residual; Prop. 1)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ke, mesh
from oracle import operator as op

Ke = ke.ke()


@pytest.mark.parametrize("dims,ndof,nfree", [
    ((16, 8, 8), 4131, 3888), ((64, 32, 32), 212355, 209088),
    ((32, 16, 16), 28611, 27744), ((48, 24, 24), 91875, 90000),
    ((96, 48, 48), 698691, 691488), ((256, 128, 128), 12830211, 12780288)])
def test_dof_counts(dims, ndof, nfree):
    nx, ny, nz = dims
    assert 3 * (nx + 1) * (ny + 1) * (nz + 1) == ndof
    assert 3 * nx * (ny + 1) * (nz + 1) == nfree
    if nx <= 64:
        g = mesh.Grid(*dims)
        assert g.n_dof == ndof and g.n_free() == nfree


def test_edge_load():
    g = mesh.Grid(6, 4, 3)
    f = g.edge_load().reshape(-1, 3)
    assert np.allclose(f.sum(axis=0), [0, 0, -1], atol=1e-15)
    nz = np.flatnonzero(np.abs(f).sum(axis=1))
    ijk = np.array([g.node_ijk(n) for n in nz])
    assert np.all(ijk[:, 0] == 6) and np.all(ijk[:, 2] == 0) and len(nz) == 5
    assert np.allclose(sorted(f[nz, 2]), [-0.25] * 3 + [-0.125] * 2)
    assert np.all(f[:, :2] == 0)


def test_young_law():
    assert op.young(np.array([0.0]), 3, 1e-3)[0] == 1e-3
    assert op.young(np.array([1.0]), 3, 1e-3)[0] == 1.0
    assert abs(op.young(np.array([0.5]), 3, 0.1)[0] - (0.1 + 0.9 * 0.125)) < 1e-16
    for bad in ([np.nan], [-0.1], [1.5]):
        with pytest.raises(ValueError):
            op.young(np.array(bad), 3, 1e-3)
    with pytest.raises(ValueError):
        op.young(np.array([0.5]), 3, 0.0)


def test_single_element_assembly_is_Ke():
    g = mesh.Grid(1, 1, 1)
    K = op.assemble(g, np.array([0.7]), Ke).toarray()
    # single element: local node a = i + 2j + 4k maps to global node i + 2j + 4k
    assert np.array_equal(K, 0.7 * Ke)


def test_two_element_bruteforce():
    g = mesh.Grid(2, 1, 1)
    E = np.array([0.3, 2.0])
    K = op.assemble(g, E, Ke).toarray()
    Kb = np.zeros((g.n_dof, g.n_dof))
    for e in range(2):
        nodes = [g.node(e + i, j, k) for (i, j, k) in ke.LOCAL]
        for a in range(8):
            for b in range(8):
                for c in range(3):
                    for d in range(3):
                        Kb[3 * nodes[a] + c, 3 * nodes[b] + d] += E[e] * Ke[3 * a + c, 3 * b + d]
    assert np.max(np.abs(K - Kb)) < 1e-15


def test_unconstrained_null_space():
    g = mesh.Grid(3, 2, 2)
    rho = np.random.default_rng(1).random(g.n_elem)
    K = op.assemble(g, op.young(rho, 3, 1e-3), Ke).toarray()
    assert np.max(np.abs(K - K.T)) <= 1e-16
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == 6


def test_prop1_floor_monotonicity():
    g = mesh.Grid(4, 3, 2)
    rho = np.random.default_rng(2).random(g.n_elem) * (np.random.default_rng(3).random(g.n_elem) > 0.4)
    p, ra, rb = 3.0, 1e-6, 1e-3
    free = g.free_dofs()
    Ka = op.free_block(op.assemble(g, op.young(rho, p, ra), Ke), free).toarray()
    Kb = op.free_block(op.assemble(g, op.young(rho, p, rb), Ke), free).toarray()
    # Prop. 1: K(rb) - K(ra) = (rb - ra) sum_e (1 - rho_e^p) K_e  (PSD)
    W = op.free_block(op.assemble(g, (rb - ra) * (1 - rho ** p), Ke), free).toarray()
    assert np.max(np.abs((Kb - Ka) - W)) <= 1e-15
    assert np.linalg.eigvalsh(Kb - Ka).min() > -1e-15
    # K(rho_min) >= rho_min K_solid
    Ks = op.free_block(op.assemble(g, np.ones(g.n_elem), Ke), free).toarray()
    assert np.linalg.eigvalsh(Ka - ra * Ks).min() > -1e-14


def test_remark_bernoulli_derivative():
    # d/drho [rho + (1-rho) rho^p] = 1 - rho^p + p (1-rho) rho^(p-1) >= 0 on (0, 1]
    for p in (3.0, 4.5):
        r = np.logspace(-12, 0, 200)
        s = lambda x: x + (1 - x) * x ** p
        h = 1e-7 * r
        fd = (s(r + h) - s(r - h)) / (2 * h)
        closed = 1 - r ** p + p * (1 - r) * r ** (p - 1)
        assert np.all(closed >= 0)
        assert np.allclose(fd, closed, rtol=1e-5, atol=1e-9)


def test_uniform_density_scales_solution():
    g = mesh.Grid(4, 2, 2)
    free = g.free_dofs()
    f = g.edge_load()[free]
    Ks = op.free_block(op.assemble(g, np.ones(g.n_elem), Ke), free)
    us = op.solve_direct(Ks, f)
    c, p, rmin = 0.37, 3.0, 1e-3
    Kc = op.free_block(op.assemble(g, op.young(np.full(g.n_elem, c), p, rmin), Ke), free)
    uc = op.solve_direct(Kc, f)
    Ec = rmin + (1 - rmin) * c ** p
    assert np.linalg.norm(uc - us / Ec) <= 1e-12 * np.linalg.norm(uc)


def test_patch_test_linear_field():
    g = mesh.Grid(4, 3, 2)
    rng = np.random.default_rng(4)
    A = rng.standard_normal((3, 3))
    t = rng.standard_normal(3)
    X = g.node_coords()
    u_lin = (X @ A.T + t).ravel()
    K = op.assemble(g, np.ones(g.n_elem), Ke).tocsr()
    i, j, k = X[:, 0], X[:, 1], X[:, 2]
    interior = (i > 0) & (i < g.nx) & (j > 0) & (j < g.ny) & (k > 0) & (k < g.nz)
    idof = np.repeat(interior, 3)
    Kii = K[idof][:, idof]
    Kib = K[idof][:, ~idof]
    ui = op.solve_direct(Kii, -(Kib @ u_lin[~idof]))
    assert np.max(np.abs(ui - u_lin[idof])) <= 1e-13 * max(1, np.abs(u_lin).max())


def test_matrix_free_and_pointwise_apply():
    g = mesh.Grid(5, 3, 4)
    rng = np.random.default_rng(5)
    E = op.young(rng.random(g.n_elem), 3, 1e-3)
    u = rng.standard_normal(g.n_dof)
    free = g.free_dofs()
    K = op.assemble(g, E, Ke)
    y_ref = np.zeros(g.n_dof)
    y_ref[free] = op.free_block(K, free) @ u[free]
    y = op.apply_full(g, E, Ke, u, chunk=7)
    assert np.max(np.abs(y - y_ref)) <= 1e-14 * np.abs(y_ref).max()
    for n in rng.integers(0, g.n_nodes, 20):
        assert np.allclose(op.apply_at_node(g, E, Ke, u, n), y_ref[3 * n:3 * n + 3], rtol=0, atol=1e-14)


def test_direct_solve_compliance_monotone_and_bounded():
    g = mesh.Grid(8, 4, 4)
    free = g.free_dofs()
    f = g.edge_load()[free]
    rho = np.random.default_rng(6).random(g.n_elem)
    Ks = op.free_block(op.assemble(g, np.ones(g.n_elem), Ke), free)
    Cs = op.compliance(f, op.solve_direct(Ks, f))
    prev = np.inf
    for rmin in (1e-9, 1e-6, 1e-4, 1e-3):
        Kf = op.free_block(op.assemble(g, op.young(rho, 3, rmin), Ke), free)
        u = op.solve_direct(Kf, f)
        assert op.relative_residual(Kf, f, u) < 1e-9
        C = op.compliance(f, u)
        assert C > 0 and Cs * (1 - 1e-12) <= C <= Cs / rmin
        assert C <= prev * (1 + 1e-9)
        prev = C
