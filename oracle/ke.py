"""Hex8 element stiffness of the unit cube (Sec. 3.1, "Discretization and units").

The paper forms one trilinear eight-node element stiffness on the reference
cube with E0 = 1, nu = 0.3 and 2x2x2 Gauss integration, and reuses it for every
element so that densities enter only through a scalar modulus.

Conventions (the paper does not state them; every test is order-invariant):
local node a = i + 2j + 4k for corner (i, j, k) in {0,1}^3, local DOF 3a + c,
element edge h = 1.

Two independent formulations are provided so each can pin the other:

* ``ke_exact``  - exact rational integration of the index form
  K[(a,i),(b,j)] = lam * int d_i N_a d_j N_b
                 + mu  * (delta_ij int grad N_a . grad N_b + int d_j N_a d_i N_b).
* ``ke_gauss``  - 2x2x2 Gauss quadrature of B^T D B in Voigt notation with
  engineering shear strains (the paper's stated rule).

The integrand is at most quadratic in each coordinate, so 2-point Gauss is exact
and the two must agree to rounding.
"""
from fractions import Fraction

import numpy as np

LOCAL = [(i, j, k) for k in (0, 1) for j in (0, 1) for i in (0, 1)]


def lame(E, nu):
    """Lame parameters of isotropic linear elasticity."""
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return lam, mu


def _factor(bit, deriv):
    """1D factor of a trilinear shape function on [0,1] as (c0, c1): c0 + c1*t.

    bit=1: t, bit=0: 1-t; deriv=True gives the derivative (a constant)."""
    if deriv:
        return (Fraction(1), Fraction(0)) if bit else (Fraction(-1), Fraction(0))
    return (Fraction(0), Fraction(1)) if bit else (Fraction(1), Fraction(-1))


def _int01(p, q):
    """Exact integral over [0,1] of (p0 + p1 t)(q0 + q1 t)."""
    return p[0] * q[0] + (p[0] * q[1] + p[1] * q[0]) / 2 + p[1] * q[1] / 3


def grad_products_exact():
    """G[a][b][d][e] = int_{[0,1]^3} dN_a/dx_d * dN_b/dx_e, exact Fractions.

    Trilinear shape functions are separable, so each integral is a product of
    three 1D integrals."""
    G = [[[[None] * 3 for _ in range(3)] for _ in range(8)] for _ in range(8)]
    for a, na in enumerate(LOCAL):
        for b, nb in enumerate(LOCAL):
            for d in range(3):
                for e in range(3):
                    val = Fraction(1)
                    for t in range(3):
                        fa = _factor(na[t], t == d)
                        fb = _factor(nb[t], t == e)
                        val *= _int01(fa, fb)
                    G[a][b][d][e] = val
    return G


def ke_exact(E=Fraction(1), nu=Fraction(3, 10)):
    """24x24 element stiffness as a list of lists of Fractions (index form)."""
    E = Fraction(E)
    nu = Fraction(nu)
    lam, mu = lame(E, nu)
    G = grad_products_exact()
    K = [[Fraction(0)] * 24 for _ in range(24)]
    for a in range(8):
        for b in range(8):
            lap = G[a][b][0][0] + G[a][b][1][1] + G[a][b][2][2]
            for i in range(3):
                for j in range(3):
                    v = lam * G[a][b][i][j] + mu * G[a][b][j][i]
                    if i == j:
                        v += mu * lap
                    K[3 * a + i][3 * b + j] = v
    return K


def ke_exact_float(E=1.0, nu=0.3):
    """Exact stiffness rounded once to FP64 (E, nu given as exact decimals)."""
    K = ke_exact(Fraction(str(E)), Fraction(str(nu)))
    return np.array([[float(v) for v in row] for row in K])


def elasticity_D(E, nu):
    """6x6 isotropic constitutive matrix, Voigt order xx, yy, zz, yz, xz, xy
    with engineering shear strains."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def ke_gauss(E=1.0, nu=0.3, npts=2):
    """Element stiffness by tensor Gauss quadrature of B^T D B (FP64)."""
    D = elasticity_D(E, nu)
    xg, wg = np.polynomial.legendre.leggauss(npts)
    xg = 0.5 * (xg + 1.0)   # map [-1,1] -> [0,1]
    wg = 0.5 * wg
    K = np.zeros((24, 24))
    for gx, wx in zip(xg, wg):
        for gy, wy in zip(xg, wg):
            for gz, wz in zip(xg, wg):
                p = (gx, gy, gz)
                B = np.zeros((6, 24))
                for a, (i, j, k) in enumerate(LOCAL):
                    f = [p[t] if bit else 1.0 - p[t] for t, bit in enumerate((i, j, k))]
                    s = [1.0 if bit else -1.0 for bit in (i, j, k)]
                    dN = (s[0] * f[1] * f[2], f[0] * s[1] * f[2], f[0] * f[1] * s[2])
                    c = 3 * a
                    B[0, c + 0] = dN[0]
                    B[1, c + 1] = dN[1]
                    B[2, c + 2] = dN[2]
                    B[3, c + 1] = dN[2]
                    B[3, c + 2] = dN[1]
                    B[4, c + 0] = dN[2]
                    B[4, c + 2] = dN[0]
                    B[5, c + 0] = dN[1]
                    B[5, c + 1] = dN[0]
                K += (wx * wy * wz) * (B.T @ D @ B)
    return K


def ke(E=1.0, nu=0.3):
    """The element stiffness used by the rest of the oracle (2x2x2 Gauss, FP64)."""
    return ke_gauss(E, nu, 2)


def hadamard8():
    """8x8 +-1 matrix whose row m holds the nodal values of the polynomial
    mode m in {1, x, y, xy, z, xz, yz, xyz} (with x -> 2i-1 etc.)."""
    H = np.zeros((8, 8))
    for a, (i, j, k) in enumerate(LOCAL):
        s = (2 * i - 1, 2 * j - 1, 2 * k - 1)
        for m in range(8):
            v = 1
            if m & 1:
                v *= s[0]
            if m & 2:
                v *= s[1]
            if m & 4:
                v *= s[2]
            H[m, a] = v
    return H


def ke_hadamard(K):
    """Ke in the per-component polynomial-mode basis: T K T^T with
    T = kron(H8, I3) (DOF 3a+c -> 3m+c)."""
    T = np.kron(hadamard8(), np.eye(3))
    return T @ K @ T.T
