"""Right-preconditioned flexible GMRES (Saad 1993) with the paper's residual
history semantics (Tab. residual-semantics; Sec. 3.5 "Why a flexible Krylov
method").

History: hist[0] = 1 (x0 = 0).  hist[k] is the estimate attached to the iterate
after k total iterations: at the start of every restart cycle it is the
recomputed true residual ||b - A x|| / ||b||; inside a cycle it is the
Givens/Hessenberg projected estimate |g_{j+1}| / ||b||.  The solve stops when
the estimate is <= tol (the paper's internal convergence flag: diagnostic
only, never an acceptance), at the iteration cap, on breakdown, or on a
non-finite value.

Readings where the paper is silent: x0 = 0; classical Gram-Schmidt with
``cgs_passes`` passes (2 = CGS2, default); the cap counts iterations across
restarts; breakdown when the new Hessenberg subdiagonal is <= 1e-14 times the
norm of the vector before orthogonalisation.
"""
import numpy as np

PROJ_CONVERGED, MAXIT, BREAKDOWN, NONFINITE = 0, 1, 2, 3


class Result:
    def __init__(self, x, hist, outcome, iters, checkpoints=()):
        self.x = x
        self.hist = np.asarray(hist)
        self.outcome = outcome
        self.iters = iters
        self.proj_eta = float(self.hist[-1])
        self.checkpoints = list(checkpoints)


def _lsq(H, g, jdone):
    """y = R^-1 g over the first jdone columns of the rotated Hessenberg."""
    y = np.zeros(jdone)
    for i in range(jdone - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:jdone] @ y[i + 1:jdone]) / H[i, i]
    return y


def fgmres(A, M, b, restart=30, max_iters=200, tol=1e-6, cgs_passes=2, breakdown=1e-14, checkpoint_every=0):
    """A, M: callables on vectors.  Returns Result.

    checkpoint_every > 0 records, after every such number of iterations, the
    recomputed true residual ||b - A x_k|| / ||b|| of the current iterate
    x_k = x + Z y_k (y_k the least-squares solution over the columns so far)
    as (k, eta) in Result.checkpoints, without changing the iteration: the
    periodic true-residual checkpoints of the probe that Sec. 4.1.1 leaves
    untested."""
    cps = []
    n = b.shape[0]
    bnorm = np.linalg.norm(b)
    x = np.zeros(n)
    hist = [1.0]
    k = 0
    if bnorm == 0.0:
        return Result(x, [0.0], PROJ_CONVERGED, 0)
    while True:
        r = b - A(x) if k > 0 else b.copy()
        beta = np.linalg.norm(r)
        if k > 0:
            hist[k] = beta / bnorm           # cycle-start true residual
        if not np.isfinite(beta):
            return Result(x, hist, NONFINITE, k, cps)
        if beta / bnorm <= tol:
            return Result(x, hist, PROJ_CONVERGED, k, cps)
        if k >= max_iters:
            return Result(x, hist, MAXIT, k, cps)
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        stop = None
        jdone = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = A(Z[j])
            wnorm0 = np.linalg.norm(w)
            h = np.zeros(j + 1)
            for _ in range(cgs_passes):
                hp = V[:j + 1] @ w
                w = w - V[:j + 1].T @ hp
                h += hp
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            if d == 0.0 or not np.isfinite(d) or not np.all(np.isfinite(h)):
                stop = NONFINITE
                jdone = j          # column j unusable
                break
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k += 1
            jdone = j + 1
            est = abs(g[j + 1]) / bnorm
            hist.append(est)
            if checkpoint_every and k % checkpoint_every == 0:
                xk = x + Z[:jdone].T @ _lsq(H, g, jdone)
                cps.append((k, float(np.linalg.norm(b - A(xk)) / bnorm)))
            if est <= tol:
                stop = PROJ_CONVERGED
            elif hn <= breakdown * wnorm0:
                stop = BREAKDOWN
            elif k >= max_iters:
                stop = MAXIT
            if stop is not None:
                break
            V[j + 1] = w / hn
        if jdone > 0:
            x = x + Z[:jdone].T @ _lsq(H, g, jdone)
        if stop is not None:
            return Result(x, hist, stop, k, cps)
