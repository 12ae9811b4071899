"""Pins of the oracle's fine-level adaptive correction (Tab. solver-config):
without inner steps it is the V-cycle; with as many inner steps as unknowns
it solves exactly; it never raises the residual of the cycle's output; and it
is homogeneous but not additive, the nonlinearity that makes the outer
method flexible (Sec. 3.5)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import adaptive as ad
from oracle import fgmres as fg
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


# ---- the rest of the adaptive stack: Chebyshev smoothing, line-searched and
# rejectable coarse correction (Tab. solver-config)

def _cheb_T(k, x):
    if abs(x) <= 1:
        return np.cos(k * np.arccos(x))
    return np.sign(x) ** k * np.cosh(k * np.arccosh(abs(x)))


@pytest.mark.parametrize("degree", [1, 2, 3, 5])
def test_chebyshev_error_polynomial(degree):
    """On K = diag(lambda_i) with B = I the Chebyshev iteration from 0 leaves
    the error p_k(K) x* with p_k(t) = T_k((c - t) / h) / T_k(c / h), the
    scaled Chebyshev polynomial of the interval [a, b]; its maximum there is
    1 / T_k(c / h) (the minimax property)."""
    lam = 2.0
    a, b = 0.1 * lam, 1.1 * lam
    c, h = 0.5 * (a + b), 0.5 * (b - a)
    t = np.concatenate([np.linspace(a, b, 40), [0.05, 1.3 * lam, 3.0]])
    K = sp.diags(t).tocsr()
    I = sp.identity(t.size, format="csr")
    xs = np.random.default_rng(degree).standard_normal(t.size)
    x = ad.chebyshev_smooth(K, I, K @ xs, np.zeros(t.size), ad.chebyshev_coefficients(lam, degree))
    p = np.array([_cheb_T(degree, (c - ti) / h) for ti in t]) / _cheb_T(degree, c / h)
    assert np.allclose(xs - x, p * xs, rtol=1e-11, atol=1e-12 * np.abs(xs).max())
    inside = (t >= a) & (t <= b)
    assert np.abs(p[inside]).max() <= 1.0 / _cheb_T(degree, c / h) * (1 + 1e-12)


def test_chebyshev_degree_one_is_the_damped_jacobi_cycle():
    """Degree 1 with the interval centred at 1 / 0.6 is one damped node-block
    Jacobi sweep (omega = 0.6): the Chebyshev V-cycle then equals the fixed
    V-cycle with one pre- and one post-sweep."""
    g = mesh.Grid(8, 4, 4)
    H = mg.build_hierarchy(g, op.young(np.random.default_rng(3).random(g.n_elem), 3.0, 1e-3), ke.ke())
    lams = [1.0 / (0.6 * 0.6)] * (len(H) - 1)        # (0.1 + 1.1) / 2 * lam = 1 / 0.6
    b = np.random.default_rng(4).standard_normal(H[0].K.shape[0])
    z1 = ad.chebyshev_vcycle(H, b, lams, nu_pre=1, nu_post=1)
    z0 = mg.vcycle(H, b, omega=0.6, nu_pre=1, nu_post=1)
    assert np.allclose(z1, z0, rtol=1e-12, atol=1e-14 * np.abs(z0).max())


def test_power_estimate_is_a_lower_bound_close_to_lambda_max():
    g = mesh.Grid(8, 4, 4)
    H = mg.build_hierarchy(g, op.young(np.random.default_rng(5).random(g.n_elem), 3.0, 1e-3), ke.ke())
    for L in H[:-1]:
        BK = (L.Binv @ L.K).toarray()
        lmax = np.max(np.linalg.eigvals(BK).real)
        est = ad.lambda_max_estimate(L.K, L.Binv, np.flatnonzero(L.grid.free_dofs()))
        assert 0.8 * lmax <= est <= lmax * (1 + 1e-12)
    # the start vector is the stated integer hash, exactly
    assert ad.hash_start([0])[0] == (0x9E3779B1 % 2 ** 32) / 2 ** 32 - 0.5
    assert ad.hash_start([2 ** 32 - 1])[0] == -0.5


def test_line_search_is_the_residual_minimizer():
    rng = np.random.default_rng(6)
    r, Kd = rng.standard_normal(50), rng.standard_normal(50)
    alpha, ratio = ad.line_search(r, Kd)
    f = lambda a: np.linalg.norm(r - a * Kd)
    assert abs((r - alpha * Kd) @ Kd) <= 1e-12 * np.linalg.norm(r) * np.linalg.norm(Kd)   # stationary
    assert f(alpha) <= min(f(alpha - 1e-3), f(alpha + 1e-3), f(0.0))
    assert ratio == pytest.approx(f(alpha) / np.linalg.norm(r), rel=1e-14) and ratio <= 1.0
    assert ad.line_search(r, np.zeros(50)) == (0.0, 1.0)


def _stack_case(dims=(16, 8, 8), seed=7, rmin=1e-3):
    # three levels: 16x8x8 (fine), 8x4x4 (600 unknowns), 4x2x2 (90, coarsest)
    g = mesh.Grid(*dims)
    H = mg.build_hierarchy(g, op.young(np.random.default_rng(seed).random(g.n_elem), 3.0, rmin), ke.ke())
    assert len(H) == 3
    v = np.random.default_rng(seed + 1).standard_normal(H[0].K.shape[0])
    return H, v


def test_rejected_coarse_correction_leaves_only_the_smoothing():
    """theta = 0 rejects every coarse correction (the ratio is never 0 here):
    the output is the Chebyshev smoothing before and after, nothing else."""
    H, v = _stack_case()
    M = ad.adaptive_stack(H, inner_steps=0, coarse_steps=4, theta=0.0)
    z = M(v)
    alpha, ratio, ok, kept = M.log[0]
    assert not ok and 0.0 < ratio < 1.0
    lam = M.lams[0]
    x = ad.chebyshev_smooth(H[0].K, H[0].Binv, v, np.zeros_like(v), ad.chebyshev_coefficients(lam, 2))
    x = ad.chebyshev_smooth(H[0].K, H[0].Binv, v, x, ad.chebyshev_coefficients(lam, 2))
    assert np.array_equal(z, x)
    # theta = 1 keeps it, scaled by the line-search step
    M1 = ad.adaptive_stack(H, inner_steps=0, coarse_steps=4, theta=1.0)
    z1 = M1(v)
    assert M1.log[0][2] and M1.log[0][0] == pytest.approx(alpha) and not np.array_equal(z1, z)
    assert np.linalg.norm(v - H[0].K @ z1) < np.linalg.norm(v - H[0].K @ z)


def test_many_coarse_steps_solve_the_coarse_problem():
    """Enough coarse GMRES steps solve the level-1 problem: the correction
    tends to P K_1^-1 P^T r, scaled by the line search (the V-cycle
    preconditioned Krylov error falls by orders of magnitude in 40 steps)."""
    H, v = _stack_case()
    M = ad.adaptive_stack(H, inner_steps=0, coarse_steps=40, theta=1.0)
    lam = ad.level_lambdas(H)
    x = ad.chebyshev_smooth(H[0].K, H[0].Binv, v, np.zeros_like(v), ad.chebyshev_coefficients(lam[0], 2))
    r = v - H[0].K @ x
    d = H[0].P @ spla.spsolve(H[1].K.tocsc(), H[0].P.T @ r)
    alpha, _ = ad.line_search(r, H[0].K @ d)
    zr = ad.chebyshev_smooth(H[0].K, H[0].Binv, v, x + alpha * d, ad.chebyshev_coefficients(lam[0], 2))
    z = M(v)
    assert np.linalg.norm(z - zr) <= 1e-8 * np.linalg.norm(zr)
    z2 = ad.adaptive_stack(H, inner_steps=0, coarse_steps=2, theta=1.0)(v)
    assert np.linalg.norm(z2 - zr) > 1e3 * np.linalg.norm(z - zr)


def test_full_stack_is_nonlinear_and_serves_flexible_gmres():
    H, v = _stack_case(seed=9, rmin=1e-6)
    M = ad.adaptive_stack(H)
    a, b = v, np.roll(v, 5)
    assert np.linalg.norm(M(2.0 * a) - 2.0 * M(a)) <= 1e-10 * np.linalg.norm(M(a))   # homogeneous
    assert np.linalg.norm(M(a + b) - M(a) - M(b)) > 1e-8 * np.linalg.norm(M(a + b))
    g = H[0].grid
    f = g.edge_load()[g.free_dofs()]
    res = fg.fgmres(lambda y: H[0].K @ y, ad.adaptive_stack(H), f, 30, 100, 1e-8)
    assert res.outcome == fg.PROJ_CONVERGED and op.relative_residual(H[0].K, f, res.x) < 1e-7
