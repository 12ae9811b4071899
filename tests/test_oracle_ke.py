"""Pins of the oracle's element stiffness against facts fixed by mathematics
(Sec. 3.1: one trilinear hex8 Ke on the unit cube, E0 = 1, nu = 0.3, 2x2x2 Gauss)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import ke

K = ke.ke()


def test_exact_matches_gauss():
    # integrand is at most quadratic per coordinate: 2-point Gauss is exact
    Kx = ke.ke_exact_float()
    assert np.max(np.abs(K - Kx)) <= 2e-16 * 4
    K3 = ke.ke_gauss(npts=3)
    assert np.max(np.abs(K - K3)) <= 1e-15


def test_lame_constants():
    lam, mu = ke.lame(Fraction(1), Fraction(3, 10))
    assert lam == Fraction(15, 26) and mu == Fraction(5, 13)


def test_exact_symmetry_and_diagonal_closed_form():
    Kx = ke.ke_exact()
    lam, mu = ke.lame(Fraction(1), Fraction(3, 10))
    # d_x N_a squared integrates to 1/9 per direction: diag = (lam + 4 mu) / 9
    for i in range(24):
        assert Kx[i][i] == (lam + 4 * mu) / 9 == Fraction(55, 234)
        for j in range(24):
            assert Kx[i][j] == Kx[j][i]
    assert sum(Kx[i][i] for i in range(24)) == Fraction(220, 39)


def _rigid_modes():
    X = np.array(ke.LOCAL, dtype=float)
    modes = []
    for c in range(3):
        t = np.zeros((8, 3))
        t[:, c] = 1.0
        modes.append(t.ravel())
    for axis in np.eye(3):
        modes.append(np.cross(axis, X).ravel())
    return np.array(modes)


def test_rigid_body_null_space_and_rank():
    R = _rigid_modes()
    assert np.max(np.abs(K @ R.T)) <= 1e-15
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-12) == 6
    assert np.linalg.matrix_rank(K, tol=1e-10) == 18
    assert ev.min() > -1e-14
    # nonzero spectrum bounds (exact values 5/78 and 5/4)
    nz = ev[np.abs(ev) > 1e-12]
    assert abs(nz.min() - 5 / 78) < 1e-13 and abs(nz.max() - 5 / 4) < 1e-13


@pytest.mark.parametrize("seed", range(5))
def test_uniform_strain_energy(seed):
    # u = eps x reproduces a uniform strain: u^T K u = lam tr(eps)^2 + 2 mu eps:eps
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3, 3))
    eps = 0.5 * (A + A.T)
    X = np.array(ke.LOCAL, dtype=float)
    u = (X @ eps.T).ravel()
    lam, mu = ke.lame(1.0, 0.3)
    energy = lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps)
    assert abs(u @ K @ u - energy) <= 1e-14 * max(1.0, energy)


def test_scaling_in_E():
    assert np.allclose(ke.ke(E=2.5), 2.5 * K, rtol=0, atol=1e-15)


def test_hadamard_structure():
    KH = ke.ke_hadamard(K)
    nz = np.abs(KH) > 1e-12
    assert nz.sum() == 45
    assert nz.sum(axis=1).max() == 3
    # the three constant modes (translations) carry no energy
    assert not nz[0:3].any() and not nz[:, 0:3].any()
