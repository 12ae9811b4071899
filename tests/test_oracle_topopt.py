"""Pins of the oracle's optimizer pieces (Sec. 3.1, Eq. to_problem, Eq.
projection; Tab. trajectory-settings): the filter against a dense matrix built
by brute force from element centres, the projection by its closed values and
finite differences, the chain rule and the full compliance gradient by
finite differences of exact solves, and the OC step by its volume constraint,
move limits, optimality relation and a closed-form special case."""
import numpy as np
import pytest

from oracle import fidelity as fd
from oracle import ke, mesh
from oracle import operator as op
from oracle import topopt as to

Ke = ke.ke()


def _dense_filter(grid, r_min):
    c = np.array([(e % grid.nx, (e // grid.nx) % grid.ny, e // (grid.nx * grid.ny))
                  for e in range(grid.n_elem)], float)
    H = np.zeros((grid.n_elem, grid.n_elem))
    for e in range(grid.n_elem):
        for j in range(grid.n_elem):
            H[e, j] = max(0.0, r_min - np.linalg.norm(c[e] - c[j]))
    return H / H.sum(axis=1, keepdims=True)


def test_linear_hat_weights_at_radius_one_and_a_half():
    offs = to.filter_offsets(1.5)
    w = sorted(round(o[3], 12) for o in offs)
    assert len(offs) == 19
    assert w.count(0.5) == 6 and w.count(1.5) == 1
    assert w.count(round(1.5 - np.sqrt(2), 12)) == 12


@pytest.mark.parametrize("dims,r", [((4, 3, 2), 1.5), ((5, 4, 3), 2.2), ((3, 1, 1), 1.5), ((2, 2, 2), 0.5)])
def test_filter_and_adjoint_equal_dense_matrix(dims, r):
    g = mesh.Grid(*dims)
    H = _dense_filter(g, r)
    rng = np.random.default_rng(1)
    x, y = rng.uniform(size=g.n_elem), rng.standard_normal(g.n_elem)
    assert np.allclose(to.density_filter(g, x, r), H @ x, rtol=1e-13, atol=1e-15)
    assert np.allclose(to.density_filter_adjoint(g, y, r), H.T @ y, rtol=1e-13, atol=1e-14)
    assert np.allclose(to.density_filter(g, np.full(g.n_elem, 0.3), r), 0.3, rtol=1e-14)


def test_projection_values_and_derivative():
    x = np.linspace(0, 1, 101)
    for beta in (1.0, 4.0, 32.0):
        p = to.project(x, beta)
        assert p[0] == pytest.approx(0.0, abs=1e-15) and p[-1] == pytest.approx(1.0, abs=1e-15)
        assert p[50] == pytest.approx(0.5, abs=1e-15)
        assert np.all(np.diff(p) > 0)
        h = 1e-6
        fdv = (to.project(x + h, beta) - to.project(x - h, beta)) / (2 * h)
        assert np.allclose(to.project_derivative(x, beta), fdv, rtol=1e-7, atol=1e-9)
    # beta -> 0: the projection tends to the identity
    assert np.allclose(to.project(x, 1e-5), x, atol=1e-9)


def test_chain_rule_through_filter_and_projection():
    g = mesh.Grid(4, 3, 2)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.2, 0.8, g.n_elem)
    a = rng.standard_normal(g.n_elem)
    F = lambda z: np.sum(a * to.physical(g, z, 1.5, 4.0) ** 2)
    grad = to.chain_to_design(g, x, 2 * a * to.physical(g, x, 1.5, 4.0), 1.5, 4.0)
    h = 1e-6
    for e in range(g.n_elem):
        d = np.zeros(g.n_elem)
        d[e] = h
        assert (F(x + d) - F(x - d)) / (2 * h) == pytest.approx(grad[e], rel=1e-6, abs=1e-10)


def _compliance(g, x, p, rmin, r, beta):
    xb = to.physical(g, x, r, beta)
    free = g.free_dofs()
    K = op.free_block(op.assemble(g, op.young(xb, p, rmin), Ke), free)
    f = g.edge_load()
    u = np.zeros(g.n_dof)
    u[free] = op.solve_direct(K, f[free])
    return fd.compliance(g, f, u), u, xb


def test_compliance_gradient_with_respect_to_the_design():
    g = mesh.Grid(4, 2, 2)
    rng = np.random.default_rng(3)
    x = rng.uniform(0.3, 0.9, g.n_elem)
    p, rmin, r, beta = 3.5, 1e-3, 1.5, 4.0
    C, u, xb = _compliance(g, x, p, rmin, r, beta)
    dcb = fd.sensitivity(xb, p, rmin, fd.element_energy(g, u, Ke))
    grad = to.chain_to_design(g, x, dcb, r, beta)
    h = 1e-6
    for e in range(g.n_elem):
        d = np.zeros(g.n_elem)
        d[e] = h
        fdv = (_compliance(g, x + d, p, rmin, r, beta)[0] - _compliance(g, x - d, p, rmin, r, beta)[0]) / (2 * h)
        assert fdv == pytest.approx(grad[e], rel=1e-5)


def test_oc_update_meets_volume_and_limits():
    g = mesh.Grid(6, 4, 3)
    rng = np.random.default_rng(4)
    x = rng.uniform(0.1, 0.6, g.n_elem)
    dc = -rng.uniform(0.01, 5.0, g.n_elem)
    beta, r, move, vf = 4.0, 1.5, 0.2, 0.3
    xt = to.density_filter(g, x, r)
    dv = to.density_filter_adjoint(g, to.project_derivative(xt, beta), r)
    xn, lam = to.oc_update(g, x, dc, dv, vf, move, r, beta)
    assert to.physical(g, xn, r, beta).sum() == pytest.approx(vf * g.n_elem, rel=1e-6)
    assert np.all(xn >= np.maximum(0, x - move) - 1e-15) and np.all(xn <= np.minimum(1, x + move) + 1e-15)
    inner = (xn > np.maximum(0, x - move) + 1e-12) & (xn < np.minimum(1, x + move) - 1e-12)
    assert inner.any()
    assert np.allclose(xn[inner], x[inner] * np.sqrt(-dc[inner] / (lam * dv[inner])), rtol=1e-12)


def test_oc_update_closed_form_without_filter_or_projection():
    # r_min < 1 keeps only the element itself, beta -> 0 makes the projection
    # linear: with uniform x and dc the step scales x to the target volume
    g = mesh.Grid(5, 3, 2)
    x = np.full(g.n_elem, 0.4)
    dc = np.full(g.n_elem, -2.0)
    dv = to.density_filter_adjoint(g, to.project_derivative(x, 1e-6), 0.5)
    xn, _ = to.oc_update(g, x, dc, dv, 0.3, 0.2, 0.5, 1e-6)
    assert np.allclose(xn, 0.3, rtol=1e-6)
