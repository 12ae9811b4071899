"""Pins of the oracle's FGMRES and history semantics (Tab. residual-semantics)
against scipy's GMRES and against exact/limit cases."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fgmres as fg
from oracle import ke, mesh
from oracle import multigrid as mg
from oracle import operator as op


def _system(dims=(8, 4, 4), seed=0, rmin=1e-3):
    g = mesh.Grid(*dims)
    free = g.free_dofs()
    E = op.young(np.random.default_rng(seed).random(g.n_elem), 3, rmin)
    K = op.free_block(op.assemble(g, E, ke.ke()), free).tocsr()
    return g, E, K, g.edge_load()[free]


def test_unpreconditioned_matches_scipy_gmres():
    g, E, K, f = _system()
    pr = []
    spla.gmres(K, f, restart=10, maxiter=3, rtol=1e-14,
               callback=lambda r: pr.append(r), callback_type="pr_norm")
    res = fg.fgmres(lambda v: K @ v, lambda v: v, f, restart=10, max_iters=30, tol=1e-14)
    assert res.iters == 30 and res.outcome == fg.MAXIT
    # inside cycles both are projected estimates; at k=10, 20 ours is the
    # recomputed true residual, equal to the projection in exact arithmetic
    assert np.allclose(res.hist[1:], pr, rtol=1e-9, atol=0)


def test_fixed_right_preconditioner_matches_gmres_on_KMinv():
    g, E, K, f = _system(seed=1)
    d = 1.0 / K.diagonal()
    Minv = lambda v: d * v
    pr = []
    KM = spla.LinearOperator(K.shape, matvec=lambda y: K @ (d * y))
    spla.gmres(KM, f, restart=15, maxiter=2, rtol=1e-14,
               callback=lambda r: pr.append(r), callback_type="pr_norm")
    res = fg.fgmres(lambda v: K @ v, Minv, f, restart=15, max_iters=30, tol=1e-14)
    assert np.allclose(res.hist[1:], pr, rtol=1e-9, atol=0)


def test_exact_preconditioner_converges_in_one_iteration():
    g, E, K, f = _system(seed=2)
    solve = spla.splu(K.tocsc()).solve
    res = fg.fgmres(lambda v: K @ v, solve, f, restart=30, max_iters=200, tol=1e-6)
    assert res.iters == 1 and res.outcome == fg.PROJ_CONVERGED
    assert op.relative_residual(K, f, res.x) < 1e-12


def test_projected_history_monotone_within_cycle_and_restart_consistency():
    g, E, K, f = _system(dims=(16, 8, 8), seed=0)
    H = mg.build_hierarchy(g, E, ke.ke())
    A = lambda v: H[0].K @ v
    M = lambda v: mg.vcycle(H, v)
    r30 = fg.fgmres(A, M, f, restart=30, max_iters=200, tol=1e-9)
    r5 = fg.fgmres(A, M, f, restart=5, max_iters=200, tol=1e-9)
    assert np.all(np.diff(r30.hist[:min(31, len(r30.hist))]) <= 1e-15)
    # identical computation up to the first restart
    assert np.array_equal(r5.hist[:5], r30.hist[:5])
    # cycle-start true residual equals the projected estimate to rounding
    assert abs(r5.hist[5] - r30.hist[5]) <= 1e-8 * r30.hist[5]
    for r in (r30, r5):
        assert r.outcome == fg.PROJ_CONVERGED
        assert op.relative_residual(H[0].K, f, r.x) < 1e-8


def test_cap_gives_visible_maxit():
    g, E, K, f = _system(seed=3)
    res = fg.fgmres(lambda v: K @ v, lambda v: v, f, restart=30, max_iters=5, tol=1e-12)
    assert res.outcome == fg.MAXIT and res.iters == 5 and len(res.hist) == 6


def test_solution_approaches_direct_solve():
    g, E, K, f = _system(dims=(16, 8, 8), seed=4)
    H = mg.build_hierarchy(g, E, ke.ke())
    u = op.solve_direct(H[0].K, f)
    res = fg.fgmres(lambda v: H[0].K @ v, lambda v: mg.vcycle(H, v), f, 30, 200, 1e-11)
    assert np.linalg.norm(res.x - u) <= 1e-7 * np.linalg.norm(u)


def test_checkpoints_equal_the_projected_estimates():
    """In exact arithmetic the projected estimate |g_{k+1}| / ||b|| is the
    residual norm of the iterate x + Z y_k, so checkpoints of the true
    residual repeat the history where the recurrence is accurate; at a
    restart boundary the checkpoint is that cycle's recomputed residual.
    The checkpoints change nothing in the iteration itself."""
    g, E, K, b = _system(seed=2)
    H = mg.build_hierarchy(g, E, ke.ke())
    A = lambda v: H[0].K @ v
    M = lambda v: mg.vcycle(H, v)
    plain = fg.fgmres(A, M, b, restart=6, max_iters=18, tol=1e-12)
    cp = fg.fgmres(A, M, b, restart=6, max_iters=18, tol=1e-12, checkpoint_every=3)
    assert np.array_equal(plain.hist, cp.hist) and np.array_equal(plain.x, cp.x)
    assert [k for k, _ in cp.checkpoints] == [3, 6, 9, 12, 15, 18][:len(cp.checkpoints)] and len(cp.checkpoints) >= 5
    for k, eta in cp.checkpoints:
        assert eta == pytest.approx(cp.hist[k], rel=1e-6)
    # unpreconditioned GMRES on the small test matrix: the same identity
    u = fg.fgmres(lambda v: K @ v, lambda v: v, b, restart=40, max_iters=40, tol=1e-14, checkpoint_every=5)
    assert len(u.checkpoints) == 8
    for k, eta in u.checkpoints:
        assert eta == pytest.approx(u.hist[k], rel=1e-8)


def test_breakdown_in_an_invariant_subspace_gives_the_exact_solution():
    """A right-hand side inside a 2-dimensional invariant subspace of A: the
    Krylov space stops growing at the second step (the subdiagonal falls to
    rounding level), the oracle exits with BREAKDOWN after 2 iterations, and
    its iterate is the exact solution (a lucky breakdown)."""
    rng = np.random.default_rng(11)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(1.0, 50.0, n)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    b = 3.0 * Q[:, 4] - 2.0 * Q[:, 17]
    res = fg.fgmres(lambda v: A @ v, lambda v: v, b, restart=30, max_iters=200, tol=0.0)
    assert res.outcome == fg.BREAKDOWN and res.iters == 2
    x = 3.0 / lam[4] * Q[:, 4] - 2.0 / lam[17] * Q[:, 17]
    assert np.linalg.norm(res.x - x) <= 1e-12 * np.linalg.norm(x)
    # with a positive tolerance the same system converges on its estimate
    res2 = fg.fgmres(lambda v: A @ v, lambda v: v, b, restart=30, max_iters=200, tol=1e-10)
    assert res2.outcome == fg.PROJ_CONVERGED and res2.iters == 2


def test_nonfinite_exits():
    """A non-finite right-hand side stops before the first step; a
    preconditioner that returns a non-finite vector stops at that step with
    the column left out, so the iterate stays the finite one of the steps
    before."""
    g, E, K, f = _system(seed=5)
    bad = f.copy()
    bad[7] = np.inf
    r = fg.fgmres(lambda v: K @ v, lambda v: v, bad, restart=10, max_iters=50, tol=1e-8)
    assert r.outcome == fg.NONFINITE and r.iters == 0 and np.all(r.x == 0)
    calls = []

    def M(v):
        calls.append(1)
        return v * np.nan if len(calls) == 4 else v
    r = fg.fgmres(lambda v: K @ v, M, f, restart=10, max_iters=50, tol=1e-12)
    ref = fg.fgmres(lambda v: K @ v, lambda v: v, f, restart=3, max_iters=3, tol=1e-12)
    assert r.outcome == fg.NONFINITE and r.iters == 3 and np.all(np.isfinite(r.x))
    # the first three steps are plain GMRES steps: same iterate as a 3-step solve
    assert np.allclose(r.x, ref.x, rtol=0, atol=1e-12 * np.abs(ref.x).max())
    assert np.array_equal(r.hist, ref.hist)
