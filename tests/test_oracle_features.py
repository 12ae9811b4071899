"""Pins of the selector's density statistics on hand-built fields."""
import numpy as np

from oracle import features


def _bar(nx=8, ny=4, nz=4, cut=None):
    rho = np.zeros((nz, ny, nx))
    rho[0, :, :] = 1.0                      # bottom layer solid from x=0 to x=L
    if cut is not None:
        rho[:, :, cut] = 0.0
    return rho.ravel()


def test_solid_bar_is_connected():
    assert features.connectivity_proxy(_bar(), 8, 4, 4) == 1.0


def test_cut_bar_is_disconnected():
    assert features.connectivity_proxy(_bar(cut=4), 8, 4, 4) == 0.0


def test_half_connected_edge():
    rho = np.zeros((4, 4, 8))
    rho[0, :2, :] = 1.0                     # only ey in {0,1} rows reach the clamp
    rho[0, 3, 6:] = 1.0                     # a loaded-edge voxel cut off by the void row ey=2
    assert features.connectivity_proxy(rho.ravel(), 8, 4, 4) == 0.5


def test_diagonal_contact_is_not_6_connected():
    rho = np.zeros((2, 2, 4))
    rho[0, 0, 0] = rho[0, 1, 1] = rho[0, 0, 2] = rho[0, 1, 3] = 1.0
    assert features.connectivity_proxy(rho.ravel(), 4, 2, 2) == 0.0


def test_density_statistics_closed_values():
    rho = np.array([0.0, 0.0, 0.5, 1.0, 0.25, 0.0, 0.75, 1.0])
    fr, mean, mn, contrast, conn, size = features.density_stats(rho, 2, 2, 2, p=3, rho0=1e-9)
    assert fr == 3 / 8 and mean == rho.mean() and mn == 0.25
    E = 1e-9 + (1 - 1e-9) * np.array([0.5, 1.0, 0.25, 0.75, 1.0]) ** 3
    assert abs(contrast - np.log10(E.max() / E.min())) < 1e-14
    assert abs(size - np.log10(81)) < 1e-15


def test_selector_features_layout():
    """Network input: log10 r50, log10 r100, then the six density statistics
    in order; a zero residual (probe converged exactly) is clamped, not -inf."""
    st = features.density_stats(np.ones(8), 2, 2, 2, 3.0, 1e-9)
    x = features.selector_features(1e-2, 1e-5, st)
    assert x[:2] == [-2.0, -5.0] and x[2:] == st and len(x) == 8
    assert features.selector_features(0.0, 1.0, st)[:2] == [-300.0, 0.0]
    assert all(np.isfinite(features.selector_features(0.0, 0.0, st)))
