"""GPU parity of the optimizer around the solve (Sec. 3.1, Eq. to_problem,
Eq. projection; Tab. trajectory-settings) against the CPU oracle, through
the C ABI: filter, adjoint, projection and the OC step on seeded inputs, the
first outer iteration against the oracle's exact solve, and the loop's
invariants in its three modes."""
import numpy as np
import pytest
import torch

from oracle import fidelity as fd
from oracle import ke as oke
from oracle import mesh
from oracle import operator as op
from oracle import topopt as to
from paper_2607_26382_amd import topoguard as tg
from paper_2607_26382_amd._lib import TopoguardError

pytestmark = pytest.mark.gpu
DEV = "cuda"
KE = oke.ke()


def _t(a):
    return torch.tensor(a, dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("dims,r", [((1, 1, 1), 1.5), ((4, 3, 2), 1.5), ((17, 9, 7), 2.2), ((6, 5, 4), 0.5),
                                    ((64, 32, 32), 1.5), ((9, 8, 7), 3.5)])
def test_filter_adjoint_projection(dims, r):
    og = mesh.Grid(*dims)
    rng = np.random.default_rng(1)
    x, a, b = rng.uniform(size=og.n_elem), rng.standard_normal(og.n_elem), rng.uniform(0.5, 2, og.n_elem)
    g = tg.Grid(*dims, max_restart=4, device=DEV)
    xt = g.density_filter(_t(x), r).cpu().numpy()
    assert np.allclose(xt, to.density_filter(og, x, r), rtol=1e-13, atol=1e-15)
    y = g.density_filter_adjoint(_t(a), _t(b), r).cpu().numpy()
    assert np.allclose(y, to.density_filter_adjoint(og, a * b, r), rtol=1e-12, atol=1e-13)
    y1 = g.density_filter_adjoint(_t(a), None, r).cpu().numpy()
    assert np.allclose(y1, to.density_filter_adjoint(og, a, r), rtol=1e-12, atol=1e-13)
    for beta in (1.0, 4.0, 32.0):
        xt2, xb, dx = (v.cpu().numpy() for v in g.filter_project(_t(x), r, beta))
        ref = to.density_filter(og, x, r)
        assert np.allclose(xt2, ref, rtol=1e-13, atol=1e-15)
        assert np.allclose(xb, to.project(ref, beta), rtol=1e-12, atol=1e-14)
        assert np.allclose(dx, to.project_derivative(ref, beta), rtol=1e-11, atol=1e-13)


def test_invalid_optimizer_arguments():
    g = tg.Grid(3, 2, 2, max_restart=4, device=DEV)
    x = _t(np.full(12, 0.3))
    with pytest.raises(TopoguardError):
        g.density_filter(x, 4.5)
    with pytest.raises(TopoguardError):
        g.filter_project(x, 1.5, beta=0.0)
    with pytest.raises(TopoguardError):
        g.oc_update(x, -x, x, 1.2, 0.2)


@pytest.mark.parametrize("dims,beta,move", [((6, 4, 3), 4.0, 0.2), ((33, 17, 9), 1.0, 0.15), ((1, 1, 1), 4.0, 0.2)])
def test_oc_update(dims, beta, move):
    og = mesh.Grid(*dims)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.1, 0.6, og.n_elem)
    dc = -rng.uniform(0.01, 5.0, og.n_elem)
    xt = to.density_filter(og, x, 1.5)
    dv = to.density_filter_adjoint(og, to.project_derivative(xt, beta), 1.5)
    vf = 0.3
    g = tg.Grid(*dims, max_restart=4, device=DEV)
    xn, lam = g.oc_update(_t(x), _t(dc), _t(dv), vf, move, 1.5, beta)
    xr, lr = to.oc_update(og, x, dc, dv, vf, move, 1.5, beta)
    # the bisections take the same steps unless a volume comparison falls
    # within rounding of the target, and then both end within 1e-9 of the root
    assert np.allclose(xn.cpu().numpy(), xr, rtol=1e-7, atol=1e-9)
    assert lam == pytest.approx(lr, rel=1e-7)


def _stage_opts(mode, max_iters, stages, tol=1e-10):
    o = tg.topopt_opts(mode=mode, max_iters=max_iters, min_iters=max_iters, stages=stages)
    o.policy.solve.tol = tol
    return o


def test_first_iteration_matches_exact_solve():
    """One outer iteration from the uniform design: the guarded solve keeps
    the original floor (uniform states are easy), and compliance and the
    OC step equal the oracle's with an exact solve (the GPU solve is taken
    to 1e-10, so its error is far below the tolerances)."""
    dims, vf, r, p, beta, move = (16, 8, 8), 0.3, 1.5, 1.5, 1.0, 0.2
    og = mesh.Grid(*dims)
    g = tg.Grid(*dims, max_restart=100, device=DEV)
    f = _t(g.edge_load())
    x0 = np.full(og.n_elem, vf)
    x1, rec = g.topopt_run(_t(x0), f, _stage_opts(tg.LOOP_GUARDED, 1, [(1, p, beta, move)]))
    assert len(rec) == 1 and rec[0]["rung"] == 0 and rec[0]["accepted"] == 1 and rec[0]["true_eta"] <= 1e-6
    # oracle: the same iteration with a direct solve at the original floor
    xb = to.physical(og, x0, r, beta)
    free = og.free_dofs()
    K = op.free_block(op.assemble(og, op.young(xb, p, 1e-12), KE), free)
    fo = og.edge_load()
    u = np.zeros(og.n_dof)
    u[free] = op.solve_direct(K, fo[free])
    C = fd.compliance(og, fo, u)
    assert rec[0]["compliance"] == pytest.approx(C, rel=1e-7)
    assert rec[0]["volume"] == pytest.approx(xb.mean(), rel=1e-12)
    dcb = fd.sensitivity(xb, p, 1e-12, fd.element_energy(og, u, KE))
    dcd = to.chain_to_design(og, x0, dcb, r, beta)
    dv = to.density_filter_adjoint(og, to.project_derivative(to.density_filter(og, x0, r), beta), r)
    xr, _ = to.oc_update(og, x0, dcd, dv, vf, move, r, beta)
    assert np.abs(x1.cpu().numpy() - xr).max() <= 1e-6
    assert np.abs(xr - x0).max() > 0.05          # the step moved the design


@pytest.mark.parametrize("mode", [tg.LOOP_GUARDED, tg.LOOP_REUSE, tg.LOOP_FIXED])
def test_loop_invariants(mode):
    dims, vf = (16, 8, 8), 0.3
    g = tg.Grid(*dims, max_restart=100, device=DEV)
    f = _t(g.edge_load())
    stages = [(1, 1.5, 1.0, 0.2), (5, 3.5, 4.0, 0.15)]
    o = tg.topopt_opts(mode=mode, max_iters=8, min_iters=8, stages=stages, fixed_floor=1e-3)
    x, rec = g.topopt_run(_t(np.full(g.n_elem, vf)), f, o)
    assert len(rec) == 8
    xn = x.cpu().numpy()
    assert np.all(xn >= 0) and np.all(xn <= 1)
    for t, r_ in enumerate(rec, 1):
        assert r_["iter"] == t and r_["p"] == (1.5 if t < 5 else 3.5) and r_["beta"] == (1.0 if t < 5 else 4.0)
        assert r_["change"] <= (0.2 if t < 5 else 0.15) + 1e-12
        assert r_["compliance"] > 0
        if t > 1 and rec[t - 2]["beta"] == r_["beta"]:
            # every OC step met the volume of the physical density (under the
            # projection it was taken with: a continuation step changes beta)
            assert r_["volume"] == pytest.approx(vf, rel=1e-6)
        if mode == tg.LOOP_FIXED:
            assert r_["accepted"] == -1 and r_["floor"] == 1e-3 and not r_["probed"]
        else:
            assert r_["accepted"] == 1 and r_["true_eta"] <= 1e-6
            assert r_["floor"] == [1e-12, 1e-3, 1e-2][r_["rung"]]
    if mode == tg.LOOP_GUARDED:
        assert all(r_["probed"] for r_ in rec)
    if mode == tg.LOOP_REUSE:
        # the probe runs at the first iteration and again only where the
        # reused floor was rejected by the guard
        assert rec[0]["probed"] and sum(r_["probed"] for r_ in rec) < len(rec)
    # deterministic: the same run again gives the same designs and records
    x2, rec2 = g.topopt_run(_t(np.full(g.n_elem, vf)), f, o)
    assert torch.equal(x, x2)
    assert [r_["compliance"] for r_ in rec] == [r_["compliance"] for r_ in rec2]
