"""Pins of the oracle's fine-level adaptive correction (Tab. solver-config):
without inner steps it is the V-cycle; with as many inner steps as unknowns
it solves exactly; it never raises the residual of the cycle's output; and it
is homogeneous but not additive, the nonlinearity that makes the outer
method flexible (Sec. 3.5)."""
import numpy as np
import pytest

from oracle import adaptive as ad
from oracle import ke, mesh
from oracle import multigrid as mg
from oracle import operator as op

Ke = ke.ke()


def _levels(dims, seed=0, rmin=1e-3, max_coarse_dof=300):
    g = mesh.Grid(*dims)
    rho = np.random.default_rng(seed).uniform(0.05, 1.0, g.n_elem)
    return mg.build_hierarchy(g, op.young(rho, 3.0, rmin), Ke, max_coarse_dof=max_coarse_dof)


def test_no_inner_steps_is_the_vcycle():
    L = _levels((8, 4, 4))
    v = np.random.default_rng(1).standard_normal(L[0].K.shape[0])
    M = ad.adaptive_preconditioner(L, 0)
    assert np.array_equal(M(v), mg.vcycle(L, v))


def test_enough_inner_steps_solve_exactly():
    # two levels on a 4x4x4 grid (300 unknowns): the cycle is inexact, the
    # inner iteration with 300 steps spans the whole space
    L = _levels((4, 4, 4), max_coarse_dof=60)
    assert len(L) == 2
    n = L[0].K.shape[0]
    v = np.random.default_rng(2).standard_normal(n)
    z = ad.adaptive_preconditioner(L, n)(v)
    x = np.linalg.solve(L[0].K.toarray(), v)
    assert np.linalg.norm(z - x) <= 1e-8 * np.linalg.norm(x)
    assert np.linalg.norm(mg.vcycle(L, v) - x) > 1e-3 * np.linalg.norm(x)


def test_correction_never_raises_the_residual():
    L = _levels((8, 4, 4), seed=3, rmin=1e-6)
    K = L[0].K
    rng = np.random.default_rng(4)
    M = ad.adaptive_preconditioner(L, 20)
    for _ in range(5):
        v = rng.standard_normal(K.shape[0])
        zv = mg.vcycle(L, v)
        assert np.linalg.norm(v - K @ M(v)) <= np.linalg.norm(v - K @ zv)
    assert all(M.log) and len(M.log) == 5


def test_homogeneous_but_not_additive():
    L = _levels((8, 4, 4), seed=5)
    rng = np.random.default_rng(6)
    a, b = rng.standard_normal((2, L[0].K.shape[0]))
    M = ad.adaptive_preconditioner(L, 20)
    assert np.allclose(M(2.5 * a), 2.5 * M(a), rtol=1e-9, atol=0)
    ab = M(a + b)
    assert np.linalg.norm(ab - (M(a) + M(b))) > 1e-6 * np.linalg.norm(ab)
