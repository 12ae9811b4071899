"""Compliance, compliance sensitivities and the operator-fidelity comparison
between floors (test infrastructure only: see the package header).

* Element strain energy e_e = u_e^T K_e u_e with u_e the element's 24 DOFs
  (clamped DOFs read as zero) and the compliance sensitivity
  dC/drho_e = -p (1 - rho_min) rho_e^(p - 1) u_e^T K_e u_e: the self-adjoint
  expression of Sec. 3.1, evaluated at the density
  rho_e that enters Eq. (floor_scaling).
* Compliance C = f^T u over the free DOFs (the normalized, dimensionless
  compliance of Sec. 3.1, "Discretization and units").
* Perturbation from a raised floor (Sec. 4.4.1, Tab. perturbation): the
  absolute relative compliance change |C_1 - C_0| / |C_0|, the relative l2
  change ||g_1 - g_0|| / ||g_0|| of the compliance gradient over the solid
  elements, and the Pearson correlation of the two gradient vectors there.
"""
import numpy as np


def element_energy(grid, u, Ke):
    """e_e = u_e^T K_e u_e for every element (FP64), clamped DOFs as zero."""
    u = np.where(grid.free_dofs(), np.asarray(u, dtype=float), 0.0)
    ue = u[grid.elem_dofs()]                       # (n_elem, 24)
    return np.einsum("ei,ij,ej->e", ue, Ke, ue)


def element_energy_at(grid, u, Ke, elems):
    """The same energies for the listed elements only, one at a time (for
    sampled checks on grids too large for the full gather)."""
    free = grid.free_dofs()
    out = np.zeros(len(elems))
    for t, e in enumerate(elems):
        ex = e % grid.nx
        ey = (e // grid.nx) % grid.ny
        ez = e // (grid.nx * grid.ny)
        ue = np.zeros(24)
        for a in range(8):
            i, j, k = ex + (a & 1), ey + ((a >> 1) & 1), ez + (a >> 2)
            n = grid.node(i, j, k)
            for c in range(3):
                ue[3 * a + c] = u[3 * n + c] if free[3 * n + c] else 0.0
        out[t] = ue @ Ke @ ue
    return out


def sensitivity(rho, p, rho_min, energy):
    """dC/drho_e = -p (1 - rho_min) rho_e^(p - 1) e_e."""
    rho = np.asarray(rho, dtype=float)
    return -p * (1.0 - rho_min) * rho ** (p - 1.0) * np.asarray(energy, dtype=float)


def compliance(grid, f, u):
    """C = f^T u over the free DOFs."""
    free = grid.free_dofs()
    return float(np.dot(np.asarray(f, dtype=float)[free], np.asarray(u, dtype=float)[free]))


def compliance_change(c0, c1):
    """|C_1 - C_0| / |C_0| (Tab. perturbation, compliance columns)."""
    return abs(c1 - c0) / abs(c0)


def gradient_change(g0, g1, solid):
    """Relative l2 change and Pearson correlation of two gradient fields over
    the elements where `solid` is True (Tab. perturbation, gradient columns).
    Pearson's r is the centred inner product over the product of the centred
    norms."""
    a = np.asarray(g0, dtype=float)[solid]
    b = np.asarray(g1, dtype=float)[solid]
    rel_l2 = float(np.linalg.norm(b - a) / np.linalg.norm(a))
    da, db = a - a.mean(), b - b.mean()
    with np.errstate(invalid="ignore", divide="ignore"):   # NaN if either field is constant
        r = float(np.dot(da, db) / np.sqrt(np.dot(da, da) * np.dot(db, db)))
    return {"n_solid": int(a.size), "rel_l2": rel_l2, "pearson": r}
