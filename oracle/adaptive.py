"""The fine-level adaptive correction of the paper's preconditioner (test
infrastructure only: see the package header).

Tab. solver-config: after the multigrid cycle, an additional correction on the
finest level, 20 steps of an inner FGMRES iteration with restart 20,
preconditioned by the 3x3 node-block Jacobi operator, applied only if it
reduces the residual norm.  With z = V(v) the cycle's output and s = v - K z,
the inner iteration solves K d = s from d = 0; z + d replaces z when
||v - K (z + d)|| < ||v - K z||.  The preconditioner so obtained depends on
its argument nonlinearly, which is why the outer method must be flexible
(Sec. 3.5).
"""
import numpy as np
import scipy.linalg as sla

from . import fgmres as fg
from . import multigrid as mg


def adaptive_preconditioner(levels, inner_steps=20):
    """v -> z: one V-cycle followed by the accepted-or-rejected fine-level
    correction.  The returned callable keeps one keep/reject flag per call in
    its attribute ``log``."""
    K = levels[0].K
    Binv = levels[0].Binv
    log = []

    def M(v):
        z = mg.vcycle(levels, v)
        if inner_steps <= 0:
            log.append(False)
            return z
        s = v - K @ z
        r0 = np.linalg.norm(s)
        inner = fg.fgmres(lambda y: K @ y, lambda y: Binv @ y, s, restart=inner_steps, max_iters=inner_steps,
                          tol=0.0)
        r1 = np.linalg.norm(s - K @ inner.x)
        ok = bool(r1 < r0)
        log.append(ok)
        return z + inner.x if ok else z

    M.log = log
    return M


# ---------------------------------------------------------------------------
# The rest of the adaptive stack of Tab. solver-config: Chebyshev smoothing
# and the line-searched, rejectable coarse-grid correction with inner Krylov
# steps on the coarse level.  Readings (the paper states none of the numbers
# below):
# * Chebyshev smoothing: the Chebyshev iteration for B^-1 K x = B^-1 b (B the
#   3 x 3 node-block diagonal of K), degree nu_pre before and nu_post after
#   the coarse correction, on the interval [lo, hi] * lambda~ with lambda~
#   ten power-iteration steps on B^-1 K from a fixed hashed start vector and
#   (lo, hi) = (0.1, 1.1);
# * coarse correction: on the finest level, after pre-smoothing with residual
#   r, the coarse problem K_1 e = P^T r gets `coarse_steps` (10) steps of
#   GMRES with restart 10 from e = 0, right-preconditioned by the Chebyshev
#   V-cycle of the levels below; the correction d = P e is scaled by the step
#   alpha that minimizes ||r - alpha K d||_2 and rejected (alpha = 0) unless
#   ||r - alpha K d|| <= theta ||r|| (acceptance ratio theta = 0.95).


def hash_start(dof_index):
    """The start vector of the power iteration: one value in [-0.5, 0.5) per
    DOF from its index d in the level's full numbering (x-fastest nodes,
    three components), ((d + 1) * 0x9E3779B1 mod 2^32) / 2^32 - 0.5; exact in
    FP64, so any implementation of the definition gives the same bits."""
    d = np.asarray(dof_index, dtype=np.uint64)
    h = ((d + np.uint64(1)) * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)
    return h.astype(np.float64) / 4294967296.0 - 0.5


def lambda_max_estimate(K, Binv, dofs, iters=10):
    """||B^-1 K v|| after `iters` power steps on B^-1 K from the hashed start
    vector (v normalized every step): an estimate of lambda_max(B^-1 K) from
    below.  dofs: the full-numbering index of every free DOF."""
    v = hash_start(dofs)
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = Binv @ (K @ v)
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam


def chebyshev_coefficients(lam, degree, lo=0.1, hi=1.1):
    """(omega_k, beta_k), k < degree, of the three-term Chebyshev step
    x_{k+1} = x_k + omega_k B^-1 (b - K x_k) + beta_k (x_k - x_{k-1}) on the
    interval [lo lam, hi lam]: with centre c = (a + b) / 2, half-width
    h = (b - a) / 2, sigma = c / h, rho_0 = 1 / sigma and
    rho_k = 1 / (2 sigma - rho_{k-1}): omega_0 = 1 / c, beta_0 = 0,
    omega_k = 2 rho_k / h, beta_k = rho_k rho_{k-1}."""
    a, b = lo * lam, hi * lam
    c, h = 0.5 * (a + b), 0.5 * (b - a)
    sigma = c / h
    out = [(1.0 / c, 0.0)]
    rho = 1.0 / sigma
    for _ in range(1, degree):
        rho_n = 1.0 / (2.0 * sigma - rho)
        out.append((2.0 * rho_n / h, rho_n * rho))
        rho = rho_n
    return out


def chebyshev_smooth(K, Binv, b, x, coefs):
    """The Chebyshev iteration from x (degree len(coefs))."""
    xp = x
    for om, be in coefs:
        xn = x + om * (Binv @ (b - K @ x)) + be * (x - xp)
        xp, x = x, xn
    return x


def level_lambdas(levels, iters=10):
    """lambda~ of every level above the coarsest."""
    out = []
    for L in levels[:-1]:
        dofs = np.flatnonzero(L.grid.free_dofs())
        out.append(lambda_max_estimate(L.K, L.Binv, dofs, iters))
    return out


def chebyshev_vcycle(levels, b, lams, nu_pre=2, nu_post=2, lo=0.1, hi=1.1, l=0):
    """The V-cycle of multigrid.vcycle with Chebyshev smoothing (degree
    nu_pre before, nu_post after the coarse correction) from level l."""
    L = levels[l]
    if L.P is None:
        return sla.cho_solve(L.chol, b)
    x = chebyshev_smooth(L.K, L.Binv, b, np.zeros_like(b), chebyshev_coefficients(lams[l], nu_pre, lo, hi))
    r = b - L.K @ x
    x = x + L.P @ chebyshev_vcycle(levels, L.P.T @ r, lams, nu_pre, nu_post, lo, hi, l + 1)
    return chebyshev_smooth(L.K, L.Binv, b, x, chebyshev_coefficients(lams[l], nu_post, lo, hi))


def line_search(r, Kd):
    """alpha minimizing ||r - alpha K d||_2 and the ratio ||r - alpha K d|| / ||r||
    (alpha = 0, ratio 1 when K d = 0)."""
    kk = float(Kd @ Kd)
    alpha = float(r @ Kd) / kk if kk > 0.0 else 0.0
    nr = np.linalg.norm(r)
    ratio = float(np.linalg.norm(r - alpha * Kd) / nr) if nr > 0.0 else 1.0
    return alpha, ratio


def adaptive_stack(levels, inner_steps=20, coarse_steps=10, theta=0.95, nu_pre=2, nu_post=2, lo=0.1, hi=1.1,
                   lams=None):
    """v -> z of the full adaptive stack: Chebyshev pre-smoothing on the finest
    level, the line-searched, rejectable coarse correction (coarse_steps of
    GMRES on level 1 preconditioned by the Chebyshev V-cycle below it; with
    coarse_steps = 0 one Chebyshev V-cycle from level 1), Chebyshev
    post-smoothing, then the fine-level correction of adaptive_preconditioner.
    The callable keeps per call (alpha, ratio, coarse accepted, fine
    correction kept) in ``log``."""
    if lams is None:
        lams = level_lambdas(levels)
    L0 = levels[0]
    K, Binv = L0.K, L0.Binv
    log = []

    def coarse(bc):
        Mc = lambda y: chebyshev_vcycle(levels, y, lams, nu_pre, nu_post, lo, hi, 1)
        if coarse_steps <= 0 or levels[1].P is None:
            return Mc(bc)
        K1 = levels[1].K
        return fg.fgmres(lambda y: K1 @ y, Mc, bc, restart=coarse_steps, max_iters=coarse_steps, tol=0.0).x

    def M(v):
        x = chebyshev_smooth(K, Binv, v, np.zeros_like(v), chebyshev_coefficients(lams[0], nu_pre, lo, hi))
        r = v - K @ x
        d = L0.P @ coarse(L0.P.T @ r)
        alpha, ratio = line_search(r, K @ d)
        ok = bool(ratio <= theta)
        if ok:
            x = x + alpha * d
        x = chebyshev_smooth(K, Binv, v, x, chebyshev_coefficients(lams[0], nu_post, lo, hi))
        kept = False
        if inner_steps > 0:
            s = v - K @ x
            inner = fg.fgmres(lambda y: K @ y, lambda y: Binv @ y, s, restart=inner_steps, max_iters=inner_steps,
                              tol=0.0)
            if np.linalg.norm(s - K @ inner.x) < np.linalg.norm(s):
                x = x + inner.x
                kept = True
        log.append((alpha, ratio, ok, kept))
        return x

    M.log = log
    M.lams = lams
    return M
