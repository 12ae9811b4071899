"""The optimizer around the state solve (test infrastructure only: see the
package header): the pieces of the minimum-compliance loop of Sec. 3.1
(Eq. to_problem) that the in-loop runs of Sec. 4.1.2 and Tab.
trajectory-settings use.

* Linear-hat density filter of radius r_min: x~_e = sum_j w_ej x_j / sum_j w_ej,
  w_ej = max(0, r_min - |c_e - c_j|) over the elements j of the grid (element
  centres on the unit lattice), and its adjoint (the chain rule through it).
* Smoothed Heaviside projection, Eq. (projection), eta = 0.5, and its
  derivative.
* Optimality-criteria update with a move limit and a bisection on the volume
  multiplier: x_new = clip(x sqrt(-dc / (lam dv)), x - move, x + move) within
  [0, 1], lam halving its bracket until sum_e xbar_e(x_new) = V* n_e
  (the volume of the physical density, Eq. to_problem).
"""
import numpy as np


def filter_offsets(r_min):
    """(dx, dy, dz, w) for every lattice offset with w = r_min - |d| > 0."""
    R = int(np.floor(r_min))
    out = []
    for dz in range(-R, R + 1):
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                w = r_min - np.sqrt(dx * dx + dy * dy + dz * dz)
                if w > 0:
                    out.append((dx, dy, dz, w))
    return out


def _shift_sum(grid, x, r_min, scale=None):
    """sum_j w_ej x_j over in-grid neighbours j of every element e (x as a
    (nz, ny, nx) array); scale, if given, multiplies x_j first."""
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    X = x.reshape(nz, ny, nx) if scale is None else (x * scale).reshape(nz, ny, nx)
    out = np.zeros((nz, ny, nx))
    for dx, dy, dz, w in filter_offsets(r_min):
        # out[e] += w * X[e + d] where both are in the grid
        zs = slice(max(0, -dz), nz - max(0, dz))
        ys = slice(max(0, -dy), ny - max(0, dy))
        xs = slice(max(0, -dx), nx - max(0, dx))
        zt = slice(max(0, dz), nz - max(0, -dz))
        yt = slice(max(0, dy), ny - max(0, -dy))
        xt = slice(max(0, dx), nx - max(0, -dx))
        out[zs, ys, xs] += w * X[zt, yt, xt]
    return out.ravel()


def filter_weight_sums(grid, r_min):
    """W_e = sum_j w_ej over the in-grid neighbours of e."""
    return _shift_sum(grid, np.ones(grid.n_elem), r_min)


def density_filter(grid, x, r_min):
    return _shift_sum(grid, np.asarray(x, dtype=float), r_min) / filter_weight_sums(grid, r_min)


def density_filter_adjoint(grid, g, r_min):
    """y_j = sum_e w_ej g_e / W_e (w symmetric, so the same stencil)."""
    W = filter_weight_sums(grid, r_min)
    return _shift_sum(grid, np.asarray(g, dtype=float) / W, r_min)


def project(xt, beta, eta=0.5):
    """Eq. (projection)."""
    xt = np.asarray(xt, dtype=float)
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return (np.tanh(beta * eta) + np.tanh(beta * (xt - eta))) / den


def project_derivative(xt, beta, eta=0.5):
    xt = np.asarray(xt, dtype=float)
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return beta * (1.0 - np.tanh(beta * (xt - eta)) ** 2) / den


def physical(grid, x, r_min, beta, eta=0.5):
    """xbar = project(filter(x))."""
    return project(density_filter(grid, x, r_min), beta, eta)


def chain_to_design(grid, x, g_phys, r_min, beta, eta=0.5):
    """d/dx of a function whose gradient with respect to xbar is g_phys."""
    xt = density_filter(grid, x, r_min)
    return density_filter_adjoint(grid, g_phys * project_derivative(xt, beta, eta), r_min)


def oc_update(grid, x, dc, dv, volfrac, move, r_min, beta, eta=0.5, rtol=1e-9, max_halvings=200):
    """One optimality-criteria step.  dc, dv: gradients of the compliance and
    of the volume sum_e xbar_e with respect to the design x.  The bracket
    [l1, l2] of the multiplier starts at [0, 1e9] and is halved while
    (l2 - l1) / (l1 + l2) > rtol: the volume at the midpoint decides which
    half is kept.  Returns (x_new, lam)."""
    x = np.asarray(x, dtype=float)
    lo = np.maximum(0.0, x - move)
    hi = np.minimum(1.0, x + move)
    ratio = np.maximum(0.0, -np.asarray(dc, dtype=float)) / np.maximum(np.asarray(dv, dtype=float), 1e-300)
    target = volfrac * grid.n_elem
    l1, l2 = 0.0, 1e9
    xn = x
    for _ in range(max_halvings):
        if (l2 - l1) / (l1 + l2) <= rtol:
            break
        lm = 0.5 * (l1 + l2)
        xn = np.clip(x * np.sqrt(ratio / lm), lo, hi)
        if physical(grid, xn, r_min, beta, eta).sum() > target:
            l1 = lm
        else:
            l2 = lm
    return xn, lm
