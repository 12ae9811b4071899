"""GPU parity of the extreme eigenvalues of K(rho_min) (Sec. 4.2) against the
oracle's ARPACK values, through the C ABI, and of the screen that the
condition number gives (Eq. screen)."""
import numpy as np
import pytest
import torch

from oracle import ke as oke
from oracle import mesh
from oracle import operator as op
from oracle import spectrum as osp
from paper_2607_26382_amd import synth
from paper_2607_26382_amd import topoguard as tg
from paper_2607_26382_amd._lib import TopoguardError

pytestmark = pytest.mark.gpu
DEV = "cuda"
KE = oke.ke()


def _field(kind, dims, seed):
    return synth.uniform(*dims, seed) if kind == "uniform" else synth.blobs(*dims, seed, blob=2)


@pytest.mark.parametrize("dims,kind,rmin,prec", [((1, 1, 1), "uniform", 1e-3, tg.F64),
                                                 ((16, 8, 8), "uniform", 1e-3, tg.F64),
                                                 ((16, 8, 8), "uniform", 1e-3, tg.BF16X3MFMA),
                                                 ((24, 12, 12), "blob", 1e-6, tg.F64),
                                                 ((24, 12, 12), "blob", 1e-6, tg.F32),
                                                 ((32, 16, 16), "blob", 1e-9, tg.BF16X3MFMA)])
def test_extreme_eigenvalues(dims, kind, rmin, prec):
    rho = _field(kind, dims, 5)
    og = mesh.Grid(*dims)
    K = op.free_block(op.assemble(og, op.young(rho, 3.0, rmin), KE), og.free_dofs())
    lmin, lmax = osp.extreme_eigenvalues(K)
    g = tg.Grid(*dims, max_restart=30, device=DEV)
    g.set_density(torch.tensor(rho, device=DEV), 3.0, rmin)
    out = g.extreme_eigenvalues(prec=prec, max_iters=400, tol=1e-7)
    assert out["converged"] == 1, out
    # Lanczos: the largest Ritz value converges to lambda_max from below
    assert out["lambda_max"] == pytest.approx(lmax, rel=1e-8) and out["lambda_max"] <= lmax * (1 + 1e-12)
    # LOBPCG: Rayleigh quotient, an upper bound on lambda_min; with the
    # residual r = ||K x - lam x|| <= 1e-7 ||K x|| its error is below r^2 / gap
    assert out["lambda_min"] == pytest.approx(lmin, rel=1e-6) and out["lambda_min"] >= lmin * (1 - 1e-9)
    kappa = lmax / lmin
    assert out["kappa"] == pytest.approx(kappa, rel=2e-6)
    assert osp.screen_floor(out["kappa"], rmin) == pytest.approx(osp.screen_floor(kappa, rmin), rel=2e-6)


def test_spectrum_needs_a_density():
    g = tg.Grid(4, 2, 2, max_restart=4, device=DEV)
    with pytest.raises(TopoguardError):
        g.extreme_eigenvalues()


def test_spectrum_is_deterministic():
    dims = (16, 8, 8)
    g = tg.Grid(*dims, max_restart=30, device=DEV)
    g.set_density(torch.tensor(synth.uniform(*dims, 1), device=DEV), 3.0, 1e-4)
    a = g.extreme_eigenvalues(prec=tg.F64)
    b = g.extreme_eigenvalues(prec=tg.F64)
    assert a == b
