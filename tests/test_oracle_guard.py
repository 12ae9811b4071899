"""Pins of the guard's evaluation in the oracle (Eq. relative_residual,
Tab. residual-semantics): the FP64 value of eta against an exactly rounded
evaluation, the rounding bound used to call an acceptance boundary-ambiguous,
the matrix-free form used at sizes that cannot be assembled, and the
degenerate right-hand sides."""
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

from oracle import ke, mesh
from oracle import operator as op

Ke = ke.ke()


def _exact_eta(grid, E, f, u):
    """eta of the operator sum_e E_e K_e (E_e and K_e entries taken as the
    exact binary rationals of their FP64 values) on free DOFs, in exact
    rational arithmetic; the square root to 40 digits."""
    free = grid.free_dofs()
    uf = [Fraction(x) if free[i] else Fraction(0) for i, x in enumerate(u)]
    y = [Fraction(0)] * grid.n_dof
    KeF = [[Fraction(x) for x in row] for row in Ke]
    for e, d in enumerate(grid.elem_dofs()):
        Ee = Fraction(E[e])
        ue = [uf[j] for j in d]
        for a in range(24):
            s = sum((KeF[a][b] * ue[b] for b in range(24)), Fraction(0))
            y[d[a]] += Ee * s
    rr = sum(((Fraction(f[i]) - y[i]) ** 2 for i in range(grid.n_dof) if free[i]), Fraction(0))
    ff = sum((Fraction(f[i]) ** 2 for i in range(grid.n_dof) if free[i]), Fraction(0))
    getcontext().prec = 40
    q = Decimal(rr.numerator) / Decimal(rr.denominator) / (Decimal(ff.numerator) / Decimal(ff.denominator))
    return float(q.sqrt())


CASES = [((2, 1, 1), 1e-3, 0), ((3, 2, 2), 1e-6, 1), ((3, 2, 2), 1e-9, 2), ((4, 2, 2), 1e-9, 3)]


@pytest.mark.parametrize("dims,rmin,seed", CASES)
def test_eta_within_bound_of_exact_value(dims, rmin, seed):
    """Near the direct solution (eta ~ 1e-16 .. 1e-7, where the rounding of
    the evaluation matters) the FP64 eta, assembled and matrix-free, lies
    within the rounding bound of the exact eta; the two bounds are valid, the
    matrix-free one no smaller than the assembled one."""
    g = mesh.Grid(*dims)
    rng = np.random.default_rng(seed)
    rho = np.where(rng.random(g.n_elem) < 0.5, 0.0, rng.uniform(0.01, 1.0, g.n_elem))
    E = op.young(rho, 3.0, rmin)
    free = g.free_dofs()
    K = op.free_block(op.assemble(g, E, Ke), free)
    f = g.edge_load()
    us = op.solve_direct(K, f[free])
    worst = 0.0
    for scale in (0.0, 1e-12, 1e-7):
        uf = us + scale * np.linalg.norm(us) * rng.standard_normal(us.size) / np.sqrt(us.size)
        u = np.zeros(g.n_dof)
        u[free] = uf
        exact = _exact_eta(g, E, f, u)
        d_asm = op.residual_bound(K, f[free], uf)
        d_mf = op.residual_bound_full(g, E, Ke, f, u)
        assert d_mf >= d_asm > 0
        e_asm = abs(op.relative_residual(K, f[free], uf) - exact)
        e_mf = abs(op.relative_residual_full(g, E, Ke, f, u) - exact)
        assert e_asm <= d_asm and e_mf <= d_mf
        worst = max(worst, e_asm, e_mf)
    if rmin <= 1e-6 and dims != (3, 2, 2) or rmin == 1e-6:
        # at low floors the evaluation error exceeds what |f| alone would
        # allow: the |K||u| term of the bound (the kappa-eps effect) is needed
        assert worst > 2 * 81 * np.finfo(float).eps


def test_matrix_free_eta_equals_assembled():
    g = mesh.Grid(8, 4, 4)
    rng = np.random.default_rng(9)
    E = op.young(rng.random(g.n_elem), 3.0, 1e-3)
    free = g.free_dofs()
    K = op.free_block(op.assemble(g, E, Ke), free)
    f = g.edge_load()
    u = rng.standard_normal(g.n_dof)
    u[~free] = 0.0
    a = op.relative_residual(K, f[free], u[free])
    b = op.relative_residual_full(g, E, Ke, f, u)
    assert abs(a - b) <= op.residual_bound(K, f[free], u[free]) + op.residual_bound_full(g, E, Ke, f, u)
    # constrained entries of u are ignored by the free-DOF operator
    u2 = u.copy()
    u2[~free] = 1e3
    assert op.relative_residual_full(g, E, Ke, f, u2) == b


def test_degenerate_right_hand_sides():
    """Eq. relative_residual is undefined for f = 0: 0 when u = 0 solves it
    exactly, NaN otherwise; a non-finite f gives NaN (never accepted)."""
    g = mesh.Grid(2, 1, 1)
    E = op.young(np.ones(g.n_elem), 3.0, 1e-3)
    free = g.free_dofs()
    K = op.free_block(op.assemble(g, E, Ke), free)
    z = np.zeros(int(free.sum()))
    assert op.relative_residual(K, z, z) == 0.0
    assert np.isnan(op.relative_residual(K, z, z + 1.0))
    f = g.edge_load()[free]
    f[0] = np.nan
    assert np.isnan(op.relative_residual(K, f, z))
    f[0] = np.inf
    assert np.isnan(op.relative_residual(K, f, z))
    assert not (np.nan <= 1e-6)
