"""Extreme eigenvalues of the frozen operator and the floor screen (test
infrastructure only: see the package header).

* lambda_min, lambda_max of the free-DOF operator K(rho_min) (Eq.
  frozen_operator), its spectral condition number kappa = lambda_max /
  lambda_min, and the indicator kappa * eps of Sec. 4.2.
* The screen of Eq. (screen): with kappa ~ c(rho) / rho_min, certification at
  tolerance tau needs rho_min >~ c(rho) eps / tau; c is taken as kappa *
  rho_min at the floor where kappa was measured.
"""
import numpy as np
import scipy.sparse.linalg as spla

EPS = np.finfo(float).eps


def extreme_eigenvalues(K_ff):
    """(lambda_min, lambda_max) of a symmetric positive definite sparse
    matrix: ARPACK on K for the largest, on K^-1 (shift-invert at 0) for the
    smallest."""
    lmax = spla.eigsh(K_ff, k=1, which="LA", return_eigenvectors=False, tol=1e-12)[0]
    lmin = spla.eigsh(K_ff, k=1, sigma=0, which="LM", return_eigenvectors=False, tol=1e-12)[0]
    return float(lmin), float(lmax)


def condition_number(K_ff):
    lmin, lmax = extreme_eigenvalues(K_ff)
    return lmax / lmin


def screen_floor(kappa, rho_min, tau=1e-6, eps=EPS):
    """Eq. (screen): c = kappa rho_min, floors below c eps / tau cannot be
    expected to certify tau."""
    return kappa * rho_min * eps / tau
