"""Pins of the oracle's extreme eigenvalues and floor screen (Sec. 4.2, Eq.
screen): dense eigenvalues on small grids, the exact scaling of the spectrum
with a uniform modulus, and the premise of the screen, kappa ~ c / rho_min
with c fixed by the field once the floor is small."""
import numpy as np
import pytest

from oracle import ke, mesh
from oracle import operator as op
from oracle import spectrum as sp
from conftest import read_table

Ke = ke.ke()


def _K(dims, rho, p, rmin):
    g = mesh.Grid(*dims)
    return op.free_block(op.assemble(g, op.young(rho, p, rmin), Ke), g.free_dofs())


@pytest.mark.parametrize("dims", [(1, 1, 1), (3, 2, 2), (4, 2, 3)])
def test_extreme_eigenvalues_equal_dense(dims):
    rng = np.random.default_rng(1)
    g = mesh.Grid(*dims)
    K = _K(dims, rng.uniform(0, 1, g.n_elem), 3.0, 1e-3)
    w = np.linalg.eigvalsh(K.toarray())
    lmin, lmax = sp.extreme_eigenvalues(K)
    assert lmin == pytest.approx(w[0], rel=1e-10) and lmax == pytest.approx(w[-1], rel=1e-12)


def test_uniform_modulus_scales_the_spectrum():
    dims = (6, 3, 3)
    g = mesh.Grid(*dims)
    a = sp.extreme_eigenvalues(_K(dims, np.ones(g.n_elem), 3.0, 1e-3))
    b = sp.extreme_eigenvalues(_K(dims, np.full(g.n_elem, 0.5), 3.0, 1e-3))
    E = 1e-3 + (1 - 1e-3) * 0.125
    assert b[0] == pytest.approx(E * a[0], rel=1e-9) and b[1] == pytest.approx(E * a[1], rel=1e-12)
    assert sp.condition_number(_K(dims, np.full(g.n_elem, 0.5), 3.0, 1e-3)) == pytest.approx(a[1] / a[0], rel=1e-9)


def test_kappa_times_floor_is_fixed_by_the_field():
    # a field with floor voids: once rho_min is small the void modes set
    # lambda_min proportional to rho_min while lambda_max stays, so
    # kappa * rho_min is nearly constant (Sec. 4.2)
    dims = (6, 3, 3)
    g = mesh.Grid(*dims)
    rng = np.random.default_rng(2)
    rho = np.where(rng.uniform(size=g.n_elem) < 0.5, 0.0, 1.0)
    c = [sp.condition_number(_K(dims, rho, 3.0, rm)) * rm for rm in (1e-8, 1e-7, 1e-6)]
    assert max(c) / min(c) < 1.01
    assert sp.screen_floor(c[0] / 1e-8, 1e-8) == pytest.approx(c[0] * np.finfo(float).eps / 1e-6)


SCREEN_ROWS = read_table("screen_cases.txt")


@pytest.mark.parametrize("row", SCREEN_ROWS, ids=[r[4][:40] for r in SCREEN_ROWS])
def test_screen_on_printed_values(row):
    """Sec. 4.2 prints kappa up to 1.6e16 at rho_0 = 1e-12 and 3.6e-6 as the
    hardest field's screen: the oracle's screen reproduces the printed value,
    and the same pair rules out half the machine epsilon and c = kappa /
    rho_min."""
    kappa, rmin, tau, want = (float(x) for x in row[:4])
    got = sp.screen_floor(kappa, rmin, tau)
    assert float(f"{got:.1e}") == want
    assert float(f"{sp.screen_floor(kappa, rmin, tau, eps=2.0 ** -53):.1e}") != want
    assert float(f"{kappa / rmin * sp.EPS / tau:.1e}") != want


def test_screen_is_where_kappa_eps_meets_tau():
    """With kappa(rho) = c / rho, the screen is the floor at which the
    indicator kappa eps equals tau (Eq. screen's derivation); floors above it
    have kappa eps < tau."""
    c, tau = 125.0, 1e-6
    s = sp.screen_floor(c / 1e-9, 1e-9, tau)
    assert (c / s) * sp.EPS == pytest.approx(tau, rel=1e-14)
    assert (c / (2 * s)) * sp.EPS < tau < (c / (0.5 * s)) * sp.EPS
