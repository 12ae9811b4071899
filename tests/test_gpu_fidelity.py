"""GPU parity of the compliance, sensitivity and gradient-comparison calls
(Sec. 3.1 sensitivity expression; Sec. 4.4.1, Tab. perturbation) against the
CPU FP64 oracle, through the C ABI.

Element by element on grids from one element to several tiles with ragged
tails and several z chunks, sampled elements at the full 256 x 128 x 128 and
64 x 32 x 32 sizes, and, end to end, the fidelity of guarded GPU solves at two
floors against the oracle's exact solves within a bound derived from the
guard tolerance and the smallest eigenvalue of K."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from oracle import fidelity as fd
from oracle import ke as oke
from oracle import mesh
from oracle import operator as op
from paper_2607_26382_amd import synth
from paper_2607_26382_amd import topoguard as tg
from paper_2607_26382_amd._lib import TopoguardError

pytestmark = pytest.mark.gpu
DEV = "cuda"
KE = oke.ke()
KE_NORM = np.linalg.norm(KE, 2)
EPS = np.finfo(float).eps


def _t(a):
    return torch.tensor(a, dtype=torch.float64, device=DEV)


def _elem_sq_norms(og, u):
    ue = np.where(og.free_dofs(), u, 0.0)[og.elem_dofs()]
    return np.einsum("ei,ei->e", ue, ue)


def _check_energy_dc(og, u, rho, p, rmin, en, dc):
    e_ref = fd.element_energy(og, u, KE)
    dc_ref = fd.sensitivity(rho, p, rmin, e_ref)
    # rounding of a 24-term quadratic form taken through the Walsh modes
    tol_e = 64 * EPS * KE_NORM * _elem_sq_norms(og, u)
    assert np.all(np.abs(en - e_ref) <= tol_e + 1e-300)
    fac = p * (1 - rmin) * rho ** (p - 1)
    assert np.all(np.abs(dc - dc_ref) <= fac * tol_e + 8 * EPS * np.abs(dc_ref) + 1e-300)


CASES = [((1, 1, 1), 3.0, 1e-3), ((3, 2, 2), 4.5, 1e-9), ((16, 8, 8), 3.0, 1e-3), ((17, 9, 7), 3.0, 1e-6),
         ((24, 12, 12), 4.5, 1e-2), ((33, 17, 5), 3.0, 1e-3), ((16, 16, 40), 3.0, 1e-3),
         ((130, 120, 41), 3.0, 1e-3), ((9, 5, 3), 3.3, 1e-3), ((7, 20, 3), 1.0, 0.0)]


@pytest.mark.parametrize("dims,p,rmin", CASES)
def test_energy_sensitivity_compliance(dims, p, rmin):
    og = mesh.Grid(*dims)
    rng = np.random.default_rng(21)
    rho = synth.uniform(*dims, 22)
    rho[rng.uniform(size=og.n_elem) < 0.3] = 0.0
    u = rng.standard_normal(og.n_dof)
    f = rng.standard_normal(og.n_dof)          # nonzero on the clamped face too: ignored
    g = tg.Grid(*dims, max_restart=4, device=DEV)
    out = g.compliance_sensitivity(_t(u), f=_t(f), rho=_t(rho), p=p, rho_min=rmin, want_energy=True)
    en, dc = out["energy"].cpu().numpy(), out["dc"].cpu().numpy()
    _check_energy_dc(og, u, rho, p, rmin, en, dc)
    free = og.free_dofs()
    c_ref = fd.compliance(og, f, u)
    assert abs(out["compliance"] - c_ref) <= og.n_free() * EPS * np.abs(f[free] * u[free]).sum()
    # fixed summation order: a second call is bitwise identical
    again = g.compliance_sensitivity(_t(u), f=_t(f), rho=_t(rho), p=p, rho_min=rmin, want_energy=True)
    assert again["compliance"] == out["compliance"]
    assert torch.equal(again["dc"], out["dc"]) and torch.equal(again["energy"], out["energy"])


def test_outputs_are_optional_and_errors_are_reported():
    dims = (5, 3, 2)
    og = mesh.Grid(*dims)
    rng = np.random.default_rng(3)
    un = rng.standard_normal(og.n_dof)
    u = _t(un)
    g = tg.Grid(*dims, max_restart=4, device=DEV)
    only_c = g.compliance_sensitivity(u, f=u)
    assert only_c["dc"] is None and only_c["energy"] is None
    assert only_c["compliance"] == pytest.approx(fd.compliance(og, un, un), rel=1e-13)
    with pytest.raises(TopoguardError):
        g.compliance_sensitivity(u)                       # nothing requested
    with pytest.raises(TopoguardError):
        g.compliance_sensitivity(u, rho=_t(np.ones(og.n_elem)), p=-1.0)
    with pytest.raises(TopoguardError):
        g.gradient_change(_t(np.zeros(og.n_elem)), u[:og.n_elem], u[:og.n_elem], solid_min=0.5)


@pytest.mark.parametrize("dims,gen", [((64, 32, 32), "severe"), ((256, 128, 128), "struts")])
def test_full_size_sampled(dims, gen):
    rho = synth.blobs(*dims, 1000) if gen == "severe" else synth.struts(*dims, 3000)
    og = mesh.Grid(*dims)
    rng = np.random.default_rng(4)
    u = rng.standard_normal(og.n_dof)
    f = og.edge_load()
    g = tg.Grid(*dims, max_restart=4, device=DEV)
    out = g.compliance_sensitivity(_t(u), f=_t(f), rho=_t(rho), p=3.0, rho_min=1e-3, want_energy=True)
    elems = np.concatenate([rng.integers(0, og.n_elem, 200), [0, og.nx - 1, og.n_elem - 1,
                                                              og.n_elem - og.nx * og.ny]])
    en = out["energy"].cpu().numpy()[elems]
    dc = out["dc"].cpu().numpy()[elems]
    e_ref = fd.element_energy_at(og, u, KE, elems)
    sq = np.array([fd.element_energy_at(og, u, np.eye(24), [e])[0] for e in elems])
    tol_e = 64 * EPS * KE_NORM * sq
    assert np.all(np.abs(en - e_ref) <= tol_e)
    dc_ref = fd.sensitivity(rho[elems], 3.0, 1e-3, e_ref)
    assert np.all(np.abs(dc - dc_ref) <= 3 * tol_e + 8 * EPS * np.abs(dc_ref) + 1e-300)
    free = og.free_dofs()
    assert abs(out["compliance"] - fd.compliance(og, f, u)) <= og.n_free() * EPS * np.abs(f[free] * u[free]).sum()


@pytest.mark.parametrize("n,frac", [(1000, 0.5), (70000, 0.3), (1, 1.0)])
def test_gradient_change(n, frac):
    # fields on a 1-D "grid" of n elements (the call reads n_elem values)
    dims = (n, 1, 1)
    rng = np.random.default_rng(5)
    rho = np.where(rng.uniform(size=n) < frac, 1.0, rng.uniform(0, 0.49, n))
    rho[0] = 1.0
    g0 = -rng.uniform(0.1, 3.0, n)
    g1 = g0 * rng.uniform(0.5, 1.5, n) + 0.01 * rng.standard_normal(n)
    g = tg.Grid(*dims, max_restart=4, device=DEV)
    out = g.gradient_change(_t(rho), _t(g0), _t(g1), solid_min=0.5)
    ref = fd.gradient_change(g0, g1, rho >= 0.5)
    assert out["n_solid"] == ref["n_solid"]
    assert out["rel_l2"] == pytest.approx(ref["rel_l2"], rel=1e-12)
    if n > 1:
        assert abs(out["pearson"] - ref["pearson"]) <= 1e-12
    s = rho >= 0.5
    assert out["norm0"] == pytest.approx(np.linalg.norm(g0[s]), rel=1e-13)
    assert out["norm1"] == pytest.approx(np.linalg.norm(g1[s]), rel=1e-13)


def _exact(og, rho, p, rmin):
    free = og.free_dofs()
    K = op.free_block(op.assemble(og, op.young(rho, p, rmin), KE), free)
    f = og.edge_load()
    u = np.zeros(og.n_dof)
    u[free] = op.solve_direct(K, f[free])
    lam_min = spla.eigsh(K, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    return u, lam_min


def test_fidelity_between_floors_matches_exact_solves():
    """Guarded GPU solves at rho_min = 1e-3 and 1e-2 on the plain 16x8x8 state:
    compliance change, gradient l2 change and correlation against the
    oracle's exact solves.  With ||f - K u|| <= tol ||f||, ||u - u*|| <=
    tol ||f|| / lambda_min(K); the element energies then move by at most
    ||Ke|| ||du_e|| (2 ||u*_e|| + ||du_e||), which bounds every metric."""
    dims, rho = synth.plain_small(0)
    og = mesh.Grid(*dims)
    p, floors, tol = 3.0, (1e-3, 1e-2), 1e-10
    g = tg.Grid(*dims, max_restart=30, device=DEV)
    f = _t(g.edge_load())
    rho_d = _t(rho)
    gpu, ref = [], []
    for rmin in floors:
        g.set_density(rho_d, p, rmin)
        u, res, _ = g.fgmres_solve(f, tg.solver_opts(tol=1e-12, max_iters=200), want_hist=False)
        assert g.true_residual(f, u) <= tol
        gpu.append(g.compliance_sensitivity(u, f=f, rho=rho_d, p=p, rho_min=rmin))
        us, lam = _exact(og, rho, p, rmin)
        fo = og.edge_load()
        du = tol * np.linalg.norm(fo) / lam                 # ||u - u*|| bound
        e_ref = fd.element_energy(og, us, KE)
        c_e = p * (1 - rmin) * rho ** (p - 1)
        # ||dg|| over all elements, each node in at most 8 elements
        B = c_e.max() * KE_NORM * du * (2 * np.sqrt(8) * np.sqrt(_elem_sq_norms(og, us).max()) + 8 * du)
        C = fd.compliance(og, fo, us)
        ref.append(dict(C=C, g=fd.sensitivity(rho, p, rmin, e_ref), B=B,
                        dC=np.linalg.norm(fo) * du + 1e-12 * C))
        assert abs(gpu[-1]["compliance"] - C) <= ref[-1]["dC"]
    solid = rho >= 0.5
    gc = g.gradient_change(rho_d, gpu[0]["dc"], gpu[1]["dc"], solid_min=0.5)
    rc = fd.gradient_change(ref[0]["g"], ref[1]["g"], solid)
    n0 = np.linalg.norm(ref[0]["g"][solid])
    B0, B1 = ref[0]["B"], ref[1]["B"]
    assert B0 < 1e-3 * n0                                  # the bound is informative here
    assert abs(gc["rel_l2"] - rc["rel_l2"]) <= (B0 + B1 + rc["rel_l2"] * B0) / (n0 - B0)
    d0 = ref[0]["g"][solid] - ref[0]["g"][solid].mean()
    d1 = ref[1]["g"][solid] - ref[1]["g"][solid].mean()
    assert abs(gc["pearson"] - rc["pearson"]) <= 2 * (B0 / np.linalg.norm(d0) + B1 / np.linalg.norm(d1))
    dC_gpu = fd.compliance_change(gpu[0]["compliance"], gpu[1]["compliance"])
    dC_ref = fd.compliance_change(ref[0]["C"], ref[1]["C"])
    assert abs(dC_gpu - dC_ref) <= 2 * (ref[0]["dC"] + ref[1]["dC"]) / ref[0]["C"]
    # every raised floor stiffens the operator: compliance decreases
    assert gpu[1]["compliance"] < gpu[0]["compliance"]
