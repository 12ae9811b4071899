"""GPU parity of the fine-level adaptive correction (Tab. solver-config) and of
the flexible GMRES around it (Sec. 3.5) against the oracle, through the C ABI:
one application on seeded vectors (the accept decision exactly, the output
element by element), zero inner steps = the V-cycle bit for bit, the outer
histories, iteration counts and per-application decisions, the mixed-precision
form judged by the FP64 guard, and the error paths."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import adaptive as oad
from oracle import fgmres as ofg
from oracle import ke as oke
from oracle import mesh
from oracle import multigrid as omg
from oracle import operator as op
from paper_2607_26382_amd import synth
from paper_2607_26382_amd import topoguard as tg
from paper_2607_26382_amd._lib import TopoguardError, lib

pytestmark = pytest.mark.gpu
DEV = "cuda"
KE = oke.ke()


def _field(kind, dims, seed):
    if kind == "uniform":
        return synth.uniform(*dims, seed)
    return synth.blobs(*dims, seed, blob=2 if kind == "blob2" else 4)


def _setup(dims, rho, rmin, max_restart=30):
    og = mesh.Grid(*dims)
    H = omg.build_hierarchy(og, op.young(rho, 3.0, rmin), KE)
    g = tg.Grid(*dims, max_restart=max_restart, device=DEV)
    g.set_density(torch.tensor(rho, dtype=torch.float64, device=DEV), 3.0, rmin)
    return og, og.free_dofs(), H, g


@pytest.mark.parametrize("dims,kind,rmin", [((16, 8, 8), "uniform", 1e-3), ((24, 12, 12), "blob", 1e-6),
                                            ((24, 12, 8), "blob2", 1e-9), ((32, 16, 16), "blob", 1e-9)])
def test_one_application_matches_oracle(dims, kind, rmin):
    rho = _field(kind, dims, 21)
    og, free, H, g = _setup(dims, rho, rmin)
    M = oad.adaptive_preconditioner(H, 20)
    rng = np.random.default_rng(8)
    for trial in range(2):
        print(f"adaptive M(v) {dims} rmin={rmin} trial {trial}", flush=True)
        v = np.zeros(og.n_dof)
        v[free] = rng.standard_normal(int(free.sum()))
        z_ref = M(v[free])
        z, acc = g.adaptive_precondition(torch.tensor(v, device=DEV), tg.F64, 20)
        z = z.cpu().numpy()
        assert acc == M.log[-1]
        assert np.all(z[~free] == 0.0)
        assert np.linalg.norm(z[free] - z_ref) <= 1e-7 * np.linalg.norm(z_ref)


def test_zero_inner_steps_is_the_vcycle():
    dims = (16, 8, 8)
    og, free, H, g = _setup(dims, synth.blobs(*dims, 4), 1e-6)
    v = np.zeros(og.n_dof)
    v[free] = np.random.default_rng(9).standard_normal(int(free.sum()))
    vt = torch.tensor(v, device=DEV)
    z, acc = g.adaptive_precondition(vt, tg.F64, 0)
    assert not acc
    assert torch.equal(z, g.vcycle(vt, tg.F64))


@pytest.mark.parametrize("dims,kind,rmin,restart", [((16, 8, 8), "uniform", 1e-3, 30),
                                                    ((16, 8, 8), "uniform", 1e-3, 1),
                                                    ((16, 8, 8), "blob", 1e-9, 7),
                                                    ((32, 16, 16), "blob", 1e-3, 30)])
def test_solve_matches_oracle(dims, kind, rmin, restart):
    rho = _field(kind, dims, 1001)
    og, free, H, g = _setup(dims, rho, rmin, max_restart=restart)
    K = H[0].K
    f_free = og.edge_load()[free]
    M = oad.adaptive_preconditioner(H, 20)
    ref = ofg.fgmres(lambda v: K @ v, M, f_free, restart, 200, 1e-6)
    print(f"adaptive FGMRES {dims} rmin={rmin} restart={restart}: oracle {ref.iters} iterations", flush=True)
    f = torch.tensor(g.edge_load(), device=DEV)
    u, res, hist, acc = g.adaptive_solve(f, tg.solver_opts(restart=restart, max_iters=200), 20)
    n = min(len(hist), len(ref.hist), 25)
    assert np.allclose(hist[:n], ref.hist[:n], rtol=1e-7, atol=0)
    assert abs(res["iterations"] - ref.iters) <= 1
    assert len(acc) == res["iterations"]
    m = min(len(acc), len(M.log), 10)
    assert acc[:m] == M.log[:m]
    assert res["outcome"] == "PROJ_CONVERGED" and ref.outcome == ofg.PROJ_CONVERGED
    eta = g.true_residual(f, u)
    assert eta <= 1e-6
    uf = u.cpu().numpy()[free]
    assert np.linalg.norm(uf - ref.x) <= 1e-5 * np.linalg.norm(ref.x)


def test_single_sweep_gram_schmidt_matches_oracle():
    dims = (16, 8, 8)
    rho = _field("blob", dims, 1001)
    og, free, H, g = _setup(dims, rho, 1e-6, max_restart=30)
    K = H[0].K
    M = oad.adaptive_preconditioner(H, 20)
    ref = ofg.fgmres(lambda v: K @ v, M, og.edge_load()[free], 30, 200, 1e-6, cgs_passes=1)
    f = torch.tensor(g.edge_load(), device=DEV)
    u, res, hist, acc = g.adaptive_solve(f, tg.solver_opts(restart=30, max_iters=200, cgs_passes=1), 20)
    n = min(len(hist), len(ref.hist), 25)
    assert np.allclose(hist[:n], ref.hist[:n], rtol=1e-7, atol=0)
    assert abs(res["iterations"] - ref.iters) <= 1
    assert acc[:10] == M.log[:10]


def test_checkpoints_match_oracle_and_leave_the_iteration_unchanged():
    dims = (16, 8, 8)
    rho = _field("blob", dims, 1001)
    og, free, H, g = _setup(dims, rho, 1e-6)
    K = H[0].K
    M = oad.adaptive_preconditioner(H, 20)
    ref = ofg.fgmres(lambda v: K @ v, M, og.edge_load()[free], 30, 200, 1e-6, checkpoint_every=4)
    f = torch.tensor(g.edge_load(), device=DEV)
    o = tg.solver_opts(restart=30, max_iters=200)
    u, res, cps = g.adaptive_checkpoints(f, o, 20, every=4)
    u2, res2, hist, acc = g.adaptive_solve(f, o, 20)
    assert torch.equal(u, u2) and res == res2
    assert len(cps) == res["iterations"] // 4 and len(cps) >= 2
    n = min(len(cps), len(ref.checkpoints))
    for (k, pj, tr), (kr, er) in zip(cps[:n], ref.checkpoints[:n]):
        assert k == kr and abs(tr - er) <= 1e-6 * er
        assert pj == hist[k]


def test_fewer_outer_iterations_than_the_plain_cycle():
    # on this state the correction is kept and cuts the outer iterations
    dims = (32, 16, 16)
    og, free, H, g = _setup(dims, synth.blobs(*dims, 1001), 1e-3)
    f = torch.tensor(g.edge_load(), device=DEV)
    o = tg.solver_opts(restart=30, max_iters=200)
    _, r0, _, a0 = g.adaptive_solve(f, o, 0)
    _, r1, _, a1 = g.adaptive_solve(f, o, 20)
    _, rf, _ = g.fgmres_solve(f, tg.solver_opts(restart=30, max_iters=200, cgs_passes=3))
    assert not any(a0)
    assert abs(r0["iterations"] - rf["iterations"]) <= 1
    assert all(a1) and r1["iterations"] < r0["iterations"]


@pytest.mark.parametrize("prec", [tg.F32, tg.BF16X3MFMA])
def test_mixed_forms_pass_the_guard(prec):
    dims = (32, 16, 16)
    og, free, H, g = _setup(dims, synth.blobs(*dims, 1001), 1e-3)
    f = torch.tensor(g.edge_load(), device=DEV)
    u, res, hist, acc = g.adaptive_solve(f, tg.solver_opts(restart=30, max_iters=200, prec=prec), 20)
    assert res["outcome"] == "PROJ_CONVERGED"
    assert g.true_residual(f, u) <= 2e-6


def test_errors():
    dims = (8, 4, 4)
    og, free, H, g = _setup(dims, synth.uniform(*dims, 0), 1e-3)
    v = torch.zeros(g.n_dof, dtype=torch.float64, device=DEV)
    z = torch.empty_like(v)
    nb = C.c_size_t()
    assert lib().tg_adaptive_workspace_bytes(g.handle, 0, 20, C.byref(nb)) == 0
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=DEV)
    ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    acc = C.c_int()
    args = (g.handle, C.c_void_p(v.data_ptr()), C.c_void_p(z.data_ptr()))
    assert lib().tg_adaptive_precondition(*args, tg.F64, 20, C.c_void_p(ptr), nb.value - 8, C.byref(acc),
                                          None) != 0
    assert lib().tg_adaptive_precondition(*args, 9, 20, C.c_void_p(ptr), nb.value, C.byref(acc), None) != 0
    assert lib().tg_adaptive_workspace_bytes(g.handle, 513, 20, C.byref(nb)) != 0
    with pytest.raises(TopoguardError):
        g.adaptive_solve(torch.tensor(g.edge_load(), device=DEV), tg.solver_opts(restart=0), 20)
    # zero right-hand side: nothing to do, zero solution
    u, res, hist, acc = g.adaptive_solve(torch.zeros_like(v), tg.solver_opts(), 20)
    assert res["iterations"] == 0 and list(hist) == [0.0] and not torch.any(u)


@pytest.mark.parametrize("prec", [tg.F64, tg.BF16X3MFMA])
def test_full_size_against_the_oracle_operator(prec):
    """The bench's workload (64x32x32 severe state, rho_min = 1e-9): a kept
    correction lowers the residual that the oracle's matrix-free FP64
    operator gives for the plain cycle's output, a rejected one leaves that
    output bit for bit; twelve flexible iterations end at a projected
    estimate equal to the oracle's recomputed residual of the iterate."""
    dims = (64, 32, 32)
    rho = synth.severe(1000)[1]
    g = tg.Grid(*dims, max_restart=30, device=DEV)
    g.set_density(torch.tensor(rho, device=DEV), 3.0, 1e-9)
    og = mesh.Grid(*dims)
    E = op.young(rho, 3.0, 1e-9)
    free = og.free_dofs()
    rng = np.random.default_rng(12)
    for trial in range(2):
        print(f"full-size adaptive M(v), prec {prec}, trial {trial}", flush=True)
        v = np.zeros(og.n_dof)
        v[free] = rng.standard_normal(int(free.sum()))
        vt = torch.tensor(v, device=DEV)
        z, acc = g.adaptive_precondition(vt, prec, 20)
        zc = g.vcycle(vt, prec) if prec == tg.F64 else g.vcycle(vt.float(), prec).double()
        z, zc = z.cpu().numpy(), zc.cpu().numpy()
        assert np.all(z[~free] == 0.0)
        if acc:
            r_kept = np.linalg.norm(v - op.apply_full(og, E, KE, z))
            r_cycle = np.linalg.norm(v - op.apply_full(og, E, KE, zc))
            assert r_kept < r_cycle
        else:
            assert np.array_equal(z, zc)
    f = og.edge_load()
    u, res, hist, acc = g.adaptive_solve(torch.tensor(f, device=DEV),
                                         tg.solver_opts(restart=30, max_iters=12, prec=prec), 20)
    assert res["iterations"] == 12 and res["outcome"] == "MAXIT" and len(acc) == 12
    eta = np.linalg.norm((f - op.apply_full(og, E, KE, u.cpu().numpy()))[free]) / np.linalg.norm(f[free])
    assert abs(eta - hist[-1]) <= 1e-6 * eta


def test_largest_restart():
    """restart = TG_AD_MAX_RESTART with no tolerance: one cycle runs until the
    estimate underflows to 0 (about 350 Arnoldi steps, so the multi-dot and
    the sweeps reach bases of over 256 vectors), following the oracle."""
    dims = (16, 8, 8)
    rho = _field("blob", dims, 7)
    og, free, H, g = _setup(dims, rho, 1e-9)
    K = H[0].K
    ref = ofg.fgmres(lambda v: K @ v, lambda v: omg.vcycle(H, v), og.edge_load()[free], 512, 512, 0.0)
    print(f"restart 512: oracle {ref.iters} iterations, outcome {ref.outcome}", flush=True)
    f = torch.tensor(g.edge_load(), device=DEV)
    u, res, hist, acc = g.adaptive_solve(f, tg.solver_opts(restart=512, max_iters=512, tol=0.0), 0)
    assert len(hist) == res["iterations"] + 1 and np.all(np.isfinite(hist))
    # at rho_min = 1e-9 the cycle's explicit coarsest inverse and the oracle's
    # Cholesky solve differ by about kappa_c eps (1e-8 relative), which the
    # early history carries at the 1e-7 level
    n = min(len(hist), len(ref.hist), 25)
    assert np.allclose(hist[:n], ref.hist[:n], rtol=1e-6, atol=0)
    assert res["outcome"] == "PROJ_CONVERGED" and ref.outcome == ofg.PROJ_CONVERGED
    assert res["iterations"] > 256 and abs(res["iterations"] - ref.iters) <= 32
    # the estimate underflows to 0 while the recomputed residual stays at this
    # operator's attainable accuracy in FP64 (about 2.6e-7 on both sides)
    ff = og.edge_load()[free]
    eta_ref = np.linalg.norm(ff - K @ ref.x) / np.linalg.norm(ff)
    eta = g.true_residual(f, u)
    assert hist[-1] == 0.0 and 0.25 * eta_ref <= eta <= 4 * eta_ref
    with pytest.raises(TopoguardError):
        g.adaptive_solve(f, tg.solver_opts(restart=513, max_iters=10), 0)
