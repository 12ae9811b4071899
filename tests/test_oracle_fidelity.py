"""Pins of the oracle's compliance, sensitivities and fidelity metrics
(Sec. 3.1 sensitivity expression; Sec. 4.4.1 and Tab. perturbation).

The element energy is pinned by closed forms of linear elasticity (a uniform
strain field and rigid motions), by the assembled operator (sum_e E_e e_e is
the quadratic form of K), by Clapeyron's identity at an exact solution, and
the sensitivity by finite differences of the compliance of exact solves.  The
comparison metrics are pinned by scaling identities, a library Pearson
routine, and the paper's own remark that a raised floor which only rescales
the (1 - rho_min) prefactor changes the gradient by exactly that factor."""
import numpy as np
import pytest
import scipy.stats

from oracle import fidelity as fd
from oracle import ke, mesh
from oracle import operator as op

Ke = ke.ke()
NU = 0.3
LAM = NU / ((1 + NU) * (1 - 2 * NU))      # Lame constants of E0 = 1, nu = 0.3
MU = 1.0 / (2 * (1 + NU))


def _linear_field(g, A, t):
    X = g.node_coords()                    # unit cubes: node (i, j, k) at (i, j, k)
    return (X @ A.T + t).ravel()


def _unclamped(g):
    return np.array([e % g.nx >= 1 for e in range(g.n_elem)])


def test_uniform_strain_energy_closed_form():
    # u = A x with A symmetric is the uniform strain eps = A; on a unit cube
    # u_e^T K_e u_e = int eps : sigma dV = lam (tr eps)^2 + 2 mu eps : eps
    rng = np.random.default_rng(3)
    g = mesh.Grid(4, 3, 2)
    B = rng.standard_normal((3, 3))
    A = 0.5 * (B + B.T)
    e = fd.element_energy(g, _linear_field(g, A, rng.standard_normal(3)), Ke)
    exact = LAM * np.trace(A) ** 2 + 2 * MU * np.sum(A * A)
    m = _unclamped(g)
    assert np.allclose(e[m], exact, rtol=1e-12, atol=0)
    # elements on the clamped face see zero displacement at their x = 0 nodes
    assert not np.allclose(e[~m], exact, rtol=1e-6)


def test_rigid_motions_store_no_energy():
    rng = np.random.default_rng(4)
    g = mesh.Grid(3, 3, 2)
    w = rng.standard_normal(3)
    W = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    u = _linear_field(g, W, rng.standard_normal(3))
    e = fd.element_energy(g, u, Ke)
    scale = np.abs(Ke).max() * np.max(np.abs(u)) ** 2
    assert np.all(np.abs(e[_unclamped(g)]) <= 1e-13 * scale)


def test_energy_sum_is_the_operator_quadratic_form():
    rng = np.random.default_rng(5)
    g = mesh.Grid(5, 3, 2)
    rho = rng.uniform(0, 1, g.n_elem)
    rho[rng.uniform(size=g.n_elem) < 0.3] = 0.0
    E = op.young(rho, 3.0, 1e-3)
    u = rng.standard_normal(g.n_dof)
    free = g.free_dofs()
    K_ff = op.free_block(op.assemble(g, E, Ke), free)
    q = u[free] @ (K_ff @ u[free])
    assert abs(np.dot(E, fd.element_energy(g, u, Ke)) - q) <= 1e-12 * abs(q)


def test_compliance_equals_stored_energy_at_the_solution():
    # Clapeyron: at K u = f, f^T u = u^T K u = sum_e E_e e_e
    rng = np.random.default_rng(6)
    g = mesh.Grid(6, 3, 3)
    rho = rng.uniform(0.05, 1, g.n_elem)
    E = op.young(rho, 3.0, 1e-3)
    free = g.free_dofs()
    K_ff = op.free_block(op.assemble(g, E, Ke), free)
    f = g.edge_load()
    u = np.zeros(g.n_dof)
    u[free] = op.solve_direct(K_ff, f[free])
    C = fd.compliance(g, f, u)
    assert C > 0
    assert abs(C - np.dot(E, fd.element_energy(g, u, Ke))) <= 1e-10 * C
    assert abs(C - op.compliance(f[free], u[free])) <= 1e-14 * C


def _exact_compliance(g, rho, p, rho_min):
    free = g.free_dofs()
    K_ff = op.free_block(op.assemble(g, op.young(rho, p, rho_min), Ke), free)
    f = g.edge_load()
    u = np.zeros(g.n_dof)
    u[free] = op.solve_direct(K_ff, f[free])
    return fd.compliance(g, f, u), u


@pytest.mark.parametrize("p,rho_min", [(3.0, 1e-3), (4.5, 1e-2)])
def test_sensitivity_matches_finite_differences(p, rho_min):
    rng = np.random.default_rng(7)
    g = mesh.Grid(3, 2, 2)
    rho = rng.uniform(0.3, 1.0, g.n_elem)
    _, u = _exact_compliance(g, rho, p, rho_min)
    sens = fd.sensitivity(rho, p, rho_min, fd.element_energy(g, u, Ke))
    assert np.all(sens < 0)
    h = 1e-5
    for e in range(g.n_elem):
        rp, rm = rho.copy(), rho.copy()
        rp[e] += h
        rm[e] -= h
        fdv = (_exact_compliance(g, rp, p, rho_min)[0] - _exact_compliance(g, rm, p, rho_min)[0]) / (2 * h)
        assert abs(fdv - sens[e]) <= 1e-6 * abs(sens[e])


def test_sensitivity_vanishes_at_zero_density():
    assert fd.sensitivity(np.array([0.0]), 3.0, 1e-3, np.array([2.0]))[0] == 0.0
    assert fd.sensitivity(np.array([1.0]), 3.0, 1e-3, np.array([2.0]))[0] == pytest.approx(-3 * 0.999 * 2)


def test_gradient_change_scaling_and_sign():
    rng = np.random.default_rng(8)
    g0 = -rng.uniform(0.1, 2.0, 500)
    solid = np.ones(500, bool)
    out = fd.gradient_change(g0, 2.5 * g0, solid)
    assert out["rel_l2"] == pytest.approx(1.5, rel=1e-14) and out["pearson"] == pytest.approx(1.0, abs=1e-14)
    out = fd.gradient_change(g0, -g0, solid)
    assert out["rel_l2"] == pytest.approx(2.0, rel=1e-14) and out["pearson"] == pytest.approx(-1.0, abs=1e-14)
    # Pearson's r is invariant under positive affine maps
    out = fd.gradient_change(g0, 3.0 * g0 + 7.0, solid)
    assert out["pearson"] == pytest.approx(1.0, abs=1e-13)


def test_pearson_matches_library():
    rng = np.random.default_rng(9)
    a = rng.standard_normal(1000)
    b = 0.3 * a + rng.standard_normal(1000)
    solid = rng.uniform(size=1000) < 0.6
    out = fd.gradient_change(a, b, solid)
    assert out["n_solid"] == solid.sum()
    assert out["pearson"] == pytest.approx(scipy.stats.pearsonr(a[solid], b[solid])[0], abs=1e-13)
    assert out["rel_l2"] == pytest.approx(np.linalg.norm(b[solid] - a[solid]) / np.linalg.norm(a[solid]), rel=1e-14)


@pytest.mark.parametrize("rho1", [1e-3, 1e-2])
def test_prefactor_alone_changes_the_gradient_by_the_floor(rho1):
    # Sec. 4.4.1: with the displacement unchanged, a raised floor enters the
    # solid-element gradient only through the (1 - rho_min) prefactor, so the
    # relative l2 change is (rho1 - rho0) / (1 - rho0), about rho1, and the
    # direction is unchanged
    rng = np.random.default_rng(10)
    rho = np.where(rng.uniform(size=400) < 0.5, 1.0, 0.0)
    e = rng.uniform(0.0, 3.0, 400)
    rho0 = 1e-12
    out = fd.gradient_change(fd.sensitivity(rho, 4.5, rho0, e), fd.sensitivity(rho, 4.5, rho1, e), rho >= 0.5)
    assert out["rel_l2"] == pytest.approx((rho1 - rho0) / (1 - rho0), rel=1e-12)
    assert out["pearson"] == pytest.approx(1.0, abs=1e-12)


def test_compliance_change():
    assert fd.compliance_change(4.0, 3.0) == 0.25
    assert fd.compliance_change(1e11, 10.0) == pytest.approx(1 - 1e-10)


def test_sampled_energies_match_the_gather():
    rng = np.random.default_rng(11)
    g = mesh.Grid(5, 4, 3)
    u = rng.standard_normal(g.n_dof)
    elems = [0, 4, 7, 19, g.n_elem - 1]
    assert np.allclose(fd.element_energy_at(g, u, Ke, elems), fd.element_energy(g, u, Ke)[elems],
                       rtol=1e-13, atol=0)
