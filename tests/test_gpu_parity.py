"""GPU parity of the HIP path against the CPU FP64 oracle, through the C ABI.

Element-by-element at sizes the oracle handles in seconds (several tiles plus
ragged tails), sampled nodes at the full workload sizes, and the edge cases
(one-element grid, grids without a direct-solvable coarsest level, invalid
input, calls out of order)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from oracle import fgmres as ofg
from oracle import ke as oke
from oracle import mesh
from oracle import multigrid as omg
from oracle import operator as op
from oracle import policy as opol
from paper_2607_26382_amd import synth
from paper_2607_26382_amd import topoguard as tg
from paper_2607_26382_amd._lib import TopoguardError

pytestmark = pytest.mark.gpu
DEV = "cuda"
KE = oke.ke()


def _case(dims, rho, p, rmin):
    og = mesh.Grid(*dims)
    free = og.free_dofs()
    E = op.young(rho, p, rmin)
    K = op.free_block(op.assemble(og, E, KE), free).tocsr()
    return og, free, E, K


def _gpu_grid(dims, rho, p, rmin, max_restart=30, mg=None):
    g = tg.Grid(*dims, max_restart=max_restart, device=DEV, mg=mg)
    g.set_density(torch.tensor(rho, dtype=torch.float64, device=DEV), p, rmin)
    return g


APPLY_CASES = [((16, 8, 8), "uniform", 1e-3), ((17, 9, 7), "uniform", 1e-3),
               ((12, 6, 6), "blob2", 1e-9), ((24, 12, 12), "blob", 1e-6), ((1, 1, 1), "uniform", 1e-3),
               ((5, 3, 2), "uniform", 1.0)]


def _field(kind, dims, seed):
    if kind == "uniform":
        return synth.uniform(*dims, seed)
    if kind == "blob2":
        return synth.blobs(*dims, seed, blob=2)
    return synth.blobs(*dims, seed, blob=4)


@pytest.mark.parametrize("dims,kind,rmin", APPLY_CASES)
def test_apply_K_f64_f32(dims, kind, rmin):
    rho = _field(kind, dims, 11)
    og, free, E, K = _case(dims, rho, 3.0, rmin)
    g = _gpu_grid(dims, rho, 3.0, rmin)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(og.n_dof)
    y_ref = np.zeros(og.n_dof)
    y_ref[free] = K @ u[free]
    bound = np.zeros(og.n_dof)
    bound[free] = abs(K) @ np.abs(u[free])
    y = g.apply_K(torch.tensor(u, device=DEV), tg.F64).cpu().numpy()
    assert np.all(np.abs(y - y_ref) <= 64 * np.finfo(float).eps * bound + 1e-300)
    assert np.all(y[~free] == 0.0)
    y32 = g.apply_K(torch.tensor(u, dtype=torch.float32, device=DEV), tg.F32).cpu().numpy()
    assert np.all(np.abs(y32 - y_ref) <= 3e-5 * bound + 1e-30)


def _oracle_vcycle(dims, rho, rmin, b_full):
    og = mesh.Grid(*dims)
    H = omg.build_hierarchy(og, op.young(rho, 3.0, rmin), KE)
    free = og.free_dofs()
    z = np.zeros(og.n_dof)
    z[free] = omg.vcycle(H, b_full[free])
    return z, H


def _solution_bound(K, ff, uf, eta):
    """||u - u*|| <= ||K^-1|| ||f - K u|| with u* the oracle's direct solve:
    the bound (eta + eta*) ||f|| / lambda_min(K), eta* the direct solve's own
    residual (triangle inequality through the exact solution)."""
    lam = spla.eigsh(K, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    us = op.solve_direct(K, ff)
    eta_s = op.relative_residual(K, ff, us)
    return np.linalg.norm(uf - us), 1.001 * (eta + eta_s) * np.linalg.norm(ff) / lam


@pytest.mark.parametrize("dims,kind,rmin", [((16, 8, 8), "uniform", 1e-3), ((32, 16, 16), "blob", 1e-9),
                                            ((17, 9, 7), "uniform", 1e-6)])
def test_true_residual_parity(dims, kind, rmin):
    """The FP64 guard against the oracle on seeded vectors: a random one and
    the oracle's exact solution plus a seeded perturbation of relative size
    1e-9 (a residual near the acceptance threshold, where the evaluation's own
    rounding matters).  Two FP64 evaluations of ||f - K u|| in different orders
    differ by at most twice n_row eps || |K||u| + |f| || / ||f||."""
    rho = _field(kind, dims, 17)
    og, free, E, K = _case(dims, rho, 3.0, rmin)
    g = _gpu_grid(dims, rho, 3.0, rmin)
    f = og.edge_load()
    ff = f[free]
    rng = np.random.default_rng(18)
    us = op.solve_direct(K, ff)
    for uf in (rng.standard_normal(ff.size), us + 1e-9 * np.linalg.norm(us) * rng.standard_normal(ff.size) / np.sqrt(ff.size)):
        u = np.zeros(og.n_dof)
        u[free] = uf
        eta = g.true_residual(torch.tensor(f, device=DEV), torch.tensor(u, device=DEV))
        assert abs(eta - op.relative_residual(K, ff, uf)) <= 2 * op.residual_bound(K, ff, uf)


# (the one-launch bottom starts at level 1 on 16x8x8, 20x8x8 and 24x12x12,
# at level 1 in FP32 and 2 in FP64 on 32x16x16, at level 2 on 48x24x24; the
# bench grid's level 3 in FP64 is covered at 64x32x32.  Coarsest inverses:
# 16x8x8 and 1x1x1 (108 and 12 free DOFs) take the register form of the
# LDS kernel, 20x8x8 (coarsest 5x2x2, 135) its LDS-resident form, 24x12x12
# (288) the global-memory kernel)
@pytest.mark.parametrize("dims,kind,rmin", [((16, 8, 8), "uniform", 1e-3), ((24, 12, 12), "blob", 1e-3),
                                            ((1, 1, 1), "uniform", 0.5), ((32, 16, 16), "blob", 1e-6),
                                            ((48, 24, 24), "blob", 1e-4), ((20, 8, 8), "blob", 1e-3)])
def test_vcycle_f64_f32(dims, kind, rmin):
    rho = _field(kind, dims, 3)
    g = _gpu_grid(dims, rho, 3.0, rmin)
    b = np.random.default_rng(1).standard_normal(g.n_dof)
    z_ref, H = _oracle_vcycle(dims, rho, rmin, b)
    assert g.n_levels == len(H)
    z = g.vcycle(torch.tensor(b, device=DEV), tg.F64).cpu().numpy()
    scale = np.abs(z_ref).max()
    assert np.abs(z - z_ref).max() <= 1e-9 * scale
    z32 = g.vcycle(torch.tensor(b, dtype=torch.float32, device=DEV), tg.F32).cpu().numpy()
    assert np.abs(z32 - z_ref).max() <= 2e-3 * scale


def test_no_vcycle_without_direct_coarsest_level():
    dims = (17, 9, 7)
    g = _gpu_grid(dims, synth.uniform(*dims, 0), 3.0, 1e-3)
    with pytest.raises(TopoguardError, match="coarsened"):
        g.vcycle(torch.zeros(g.n_dof, dtype=torch.float64, device=DEV))


def _oracle_fgmres(dims, rho, rmin, restart, cap, tol=1e-6):
    og = mesh.Grid(*dims)
    H = omg.build_hierarchy(og, op.young(rho, 3.0, rmin), KE)
    f = og.edge_load()[og.free_dofs()]
    res = ofg.fgmres(lambda v: H[0].K @ v, lambda v: omg.vcycle(H, v), f, restart, cap, tol)
    return res, H, f, og


@pytest.mark.parametrize("cgs", [2, 3])
@pytest.mark.parametrize("dims,kind,rmin,restart", [((16, 8, 8), "uniform", 1e-3, 30),
                                                    ((16, 8, 8), "uniform", 1e-3, 7),
                                                    ((32, 16, 16), "blob", 1e-4, 30)])
def test_fgmres_history_and_solution(dims, kind, rmin, restart, cgs):
    """Both CGS2 forms (reorthogonalization delayed into the next step, or in
    place) follow the oracle's FGMRES (Saad, CGS2)."""
    rho = _field(kind, dims, 1001)
    ref, H, f_free, og = _oracle_fgmres(dims, rho, rmin, restart, 200)
    g = _gpu_grid(dims, rho, 3.0, rmin)
    f = torch.tensor(g.edge_load(), device=DEV)
    u, res, hist = g.fgmres_solve(f, tg.solver_opts(restart=restart, cgs_passes=cgs))
    n = min(len(hist), len(ref.hist), 25)
    assert np.allclose(hist[:n], ref.hist[:n], rtol=1e-8, atol=0)
    assert abs(res["iterations"] - ref.iters) <= 1
    assert res["outcome"] == "PROJ_CONVERGED" and ref.outcome == ofg.PROJ_CONVERGED
    assert g.true_residual(f, u) <= 1e-6
    uf = u.cpu().numpy()[og.free_dofs()]
    assert np.linalg.norm(uf - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_one_element_grid_solves_in_one_iteration():
    dims = (1, 1, 1)
    g = _gpu_grid(dims, np.array([0.7]), 3.0, 1e-3)
    f = torch.tensor(g.edge_load(), device=DEV)
    u, res, hist = g.fgmres_solve(f, tg.solver_opts())
    assert res["iterations"] == 1 and g.true_residual(f, u) < 1e-12


def test_cap_gives_visible_maxit():
    dims = (16, 8, 8)
    g = _gpu_grid(dims, synth.uniform(*dims, 0), 3.0, 1e-3)
    f = torch.tensor(g.edge_load(), device=DEV)
    u, res, hist = g.fgmres_solve(f, tg.solver_opts(max_iters=5, tol=1e-12))
    assert res["outcome"] == "MAXIT" and res["iterations"] == 5 and len(hist) == 6


def test_probe_features_match_oracle():
    dims = (32, 16, 16)
    rho = synth.blobs(*dims, 1001)
    ref, H, f_free, og = _oracle_fgmres(dims, rho, 1e-9, 100, 100)
    r50_o, r100_o = opol.probe_features(ref.hist, ref.iters)
    g = _gpu_grid(dims, rho, 3.0, 1e-9, max_restart=100)
    f = torch.tensor(g.edge_load(), device=DEV)
    r50, r100, ks = g.probe_features(f, 100, 100)
    assert ks == ref.iters
    assert abs(r50 - r50_o) <= 1e-6 * r50_o and abs(r100 - r100_o) <= 1e-6 * r100_o


def _oracle_select(dims, rho, rungs, restart=30, cap=200):
    og = mesh.Grid(*dims)
    free = og.free_dofs()
    f = og.edge_load()[free]
    cache = {}

    def hier(fl):
        if fl not in cache:
            cache[fl] = omg.build_hierarchy(og, op.young(rho, 3.0, fl), KE)
        return cache[fl]

    def probe(fl):
        H = hier(fl)
        r = ofg.fgmres(lambda v: H[0].K @ v, lambda v: omg.vcycle(H, v), f, 100, 100, 1e-6)
        return r.hist, r.iters

    def solve(fl):
        H = hier(fl)
        r = ofg.fgmres(lambda v: H[0].K @ v, lambda v: omg.vcycle(H, v), f, restart, cap, 1e-6)
        return r.x, r.iters, r.outcome, r.proj_eta

    def eta(fl, u):
        return op.relative_residual(hier(fl)[0].K, f, u)

    return opol.select_floor(rungs, probe, solve, eta)


@pytest.mark.parametrize("seed", [1000, 1001])
def test_select_floor_matches_oracle(seed):
    dims = (32, 16, 16)
    rho = synth.blobs(*dims, seed)
    rungs = [1e-9, 1e-6, 1e-4, 1e-3]
    ref = _oracle_select(dims, rho, rungs)
    g = tg.Grid(*dims, max_restart=100, device=DEV)
    f = torch.tensor(g.edge_load(), device=DEV)
    rho_d = torch.tensor(rho, device=DEV)
    u, out = g.select_floor(rho_d, f, tg.policy(rungs=rungs))
    assert out["k0"] == ref["k0"]
    assert abs(out["r50"] - ref["r50"]) <= 1e-6 * ref["r50"]
    assert out["rung"] == ref["rung"]
    assert [a["rung"] for a in out["attempts"]] == [a.rung for a in ref["attempts"]]
    for a, b in zip(out["attempts"], ref["attempts"]):
        assert abs(a["iterations"] - b.iters) <= 1
        assert a["accepted"] == b.accepted
    if out["rung"] >= 0:
        # the accepted solution passed the FP64 guard (whose parity with the
        # oracle is tested on seeded vectors in test_true_residual_parity)
        assert out["attempts"][-1]["accepted"] and out["attempts"][-1]["true_eta"] <= 1e-6
        assert g.true_residual(f, u) <= 1e-6


def test_batch_equals_individual_solves():
    dims_list = [(16, 8, 8), (24, 12, 12), (16, 8, 8)]
    rhos = [synth.uniform(*dims_list[0], 0), synth.blobs(*dims_list[1], 7), synth.uniform(*dims_list[2], 9)]
    floors = [1e-3, 1e-4, 1e-2]
    grids = [tg.Grid(*d, max_restart=30, device=DEV) for d in dims_list]
    batch = tg.Batch(grids)
    rho_d = [torch.tensor(r, device=DEV) for r in rhos]
    batch.set_density(rho_d, 3.0, floors)
    fs = [torch.tensor(g.edge_load(), device=DEV) for g in grids]
    us, res = batch.solve(fs)
    for i, d in enumerate(dims_list):
        g1 = _gpu_grid(d, rhos[i], 3.0, floors[i])
        u1, r1, _ = g1.fgmres_solve(fs[i])
        assert r1["iterations"] == res[i]["iterations"]
        assert torch.equal(u1, us[i])            # deterministic reductions: bitwise equal
        assert res[i]["true_eta"] <= 1e-6


def test_invalid_density_and_order_errors():
    dims = (8, 4, 4)
    g = tg.Grid(*dims, device=DEV)
    u = torch.zeros(g.n_dof, dtype=torch.float64, device=DEV)
    with pytest.raises(TopoguardError, match="set_density"):
        g.apply_K(u)
    bad = torch.full((g.n_elem,), 0.5, dtype=torch.float64, device=DEV)
    bad[3] = float("nan")
    with pytest.raises(TopoguardError, match="density"):
        g.set_density(bad, 3.0, 1e-3)
    bad[3] = 1.5
    with pytest.raises(TopoguardError, match="density"):
        g.set_density(bad, 3.0, 1e-3)
    with pytest.raises(TopoguardError, match="rho_min"):
        g.set_density(torch.full((g.n_elem,), 0.5, dtype=torch.float64, device=DEV), 3.0, 0.0)


@pytest.mark.parametrize("dims,gen", [((64, 32, 32), "severe"), ((256, 128, 128), "struts")])
def test_full_size_apply_sampled(dims, gen):
    rho = synth.blobs(*dims, 1000) if gen == "severe" else synth.struts(*dims, 3000)
    rmin = 1e-9 if gen == "severe" else 1e-3
    g = tg.Grid(*dims, max_restart=4, device=DEV)
    g.set_density(torch.tensor(rho, device=DEV), 3.0, rmin)
    og = mesh.Grid(*dims)
    E = op.young(rho, 3.0, rmin)
    rng = np.random.default_rng(2)
    u = rng.standard_normal(og.n_dof)
    y = g.apply_K(torch.tensor(u, device=DEV), tg.F64).cpu().numpy()
    u32 = torch.tensor(u, dtype=torch.float32, device=DEV)
    y32 = g.apply_K(u32, tg.F32).cpu().numpy()
    y3 = g.apply_K(u32, tg.BF16X3MFMA).cpu().numpy()
    nodes = np.concatenate([rng.integers(0, og.n_nodes, 150),
                            [0, og.n_nodes - 1, og.node(og.nx, og.ny, 0), og.node(1, 0, og.nz)]])
    Ka = np.abs(KE)
    for n in nodes:
        ref = op.apply_at_node(og, E, KE, u, int(n))
        bnd = op.apply_at_node(og, E, Ka, np.abs(u), int(n))
        assert np.all(np.abs(y[3 * n:3 * n + 3] - ref) <= 64 * 2.2e-16 * bnd + 1e-300)
        assert np.all(np.abs(y32[3 * n:3 * n + 3] - ref) <= 3e-5 * bnd + 1e-30)
        assert np.all(np.abs(y3[3 * n:3 * n + 3] - ref) <= 2.0 ** -13 * bnd + 1e-30)


@pytest.mark.parametrize("dims,kind,rmin", [((16, 8, 8), "uniform", 1e-3), ((32, 16, 16), "blob", 1e-4),
                                            ((32, 16, 16), "blob", 1e-9)])
def test_mixed_precision_solve_certified_by_oracle(dims, kind, rmin):
    """FP32 V-cycle inside FP64 FGMRES: the result is judged only by the FP64
    residual, recomputed here by the oracle; it must approach the FP64 solve."""
    rho = _field(kind, dims, 1001)
    og = mesh.Grid(*dims)
    free = og.free_dofs()
    K = op.free_block(op.assemble(og, op.young(rho, 3.0, rmin), KE), free)
    ff = og.edge_load()[free]
    g = _gpu_grid(dims, rho, 3.0, rmin)
    f = torch.tensor(g.edge_load(), device=DEV)
    u32, r32, h32 = g.fgmres_solve(f, tg.solver_opts(prec=tg.F32))
    u64, r64, h64 = g.fgmres_solve(f, tg.solver_opts(prec=tg.F64))
    eta32 = g.true_residual(f, u32)
    if eta32 <= 1e-6:
        # ||u - u*|| <= ||K^-1|| ||f - K u|| against the oracle's exact solve
        err, bnd = _solution_bound(K, ff, u32.cpu().numpy()[free], eta32)
        assert err <= bnd
    if r32["outcome"] == "PROJ_CONVERGED" and eta32 <= 1e-6:
        # both accepted: the two solutions agree to the conditioning of the solve
        d = np.linalg.norm((u32 - u64).cpu().numpy()) / np.linalg.norm(u64.cpu().numpy())
        assert d < 1e-2
    # iteration counts stay close to the FP64 solve on these fields
    assert r32["iterations"] <= r64["iterations"] + 10


def test_mixed_policy_matches_oracle_rungs():
    dims = (32, 16, 16)
    rungs = [1e-9, 1e-6, 1e-4, 1e-3]
    for seed in (1000, 1001):
        rho = synth.blobs(*dims, seed)
        ref = _oracle_select(dims, rho, rungs)
        g = tg.Grid(*dims, max_restart=100, device=DEV)
        f = torch.tensor(g.edge_load(), device=DEV)
        pol = tg.policy(rungs=rungs, solve=tg.solver_opts(prec=tg.F32))
        u, out = g.select_floor(torch.tensor(rho, device=DEV), f, pol)
        assert out["rung"] == ref["rung"]
        g.set_density(torch.tensor(rho, device=DEV), 3.0, rungs[out["rung"]])
        assert out["attempts"][-1]["true_eta"] <= 1e-6 and g.true_residual(f, u) <= 1e-6


@pytest.mark.parametrize("dims,kind,rmin", [((16, 8, 8), "uniform", 1e-3), ((17, 9, 7), "uniform", 1e-3),
                                            ((24, 12, 12), "blob", 1e-6)])
def test_apply_K_bf16_matrix_cores(dims, kind, rmin):
    """BF16 inputs (u and Ke rounded to 8-bit significands) with FP32
    accumulation: each product is off by at most ~2^-8 relative twice, so
    |y - y_ref| <= 2^-7 (|K||u|); split BF16 keeps ~16 bits: 2^-13 (|K||u|)."""
    rho = _field(kind, dims, 11)
    og, free, E, K = _case(dims, rho, 3.0, rmin)
    g = _gpu_grid(dims, rho, 3.0, rmin)
    u = np.random.default_rng(5).standard_normal(og.n_dof)
    y_ref = np.zeros(og.n_dof)
    y_ref[free] = K @ u[free]
    bound = np.zeros(og.n_dof)
    bound[free] = abs(K) @ np.abs(u[free])
    ut = torch.tensor(u, dtype=torch.float32, device=DEV)
    y1 = g.apply_K(ut, tg.BF16MFMA).cpu().numpy()
    y3 = g.apply_K(ut, tg.BF16X3MFMA).cpu().numpy()
    assert np.all(np.abs(y1 - y_ref) <= 2.0 ** -7 * bound + 1e-30)
    assert np.all(np.abs(y3 - y_ref) <= 2.0 ** -13 * bound + 1e-30)
    assert np.all(y1[~free] == 0) and np.all(y3[~free] == 0)
    # the BF16 result is not the FP32 result: the matrix cores really ran
    y32 = g.apply_K(ut, tg.F32).cpu().numpy()
    assert np.abs(y1 - y32).max() > 0


@pytest.mark.parametrize("prec", ["BF16MFMA", "BF16X3MFMA"])
def test_bf16_vcycle_and_solve_certified(prec):
    """Plain BF16 rounds Ke, which breaks its exact rigid-body null space: on
    high-contrast states the preconditioner may then stall.  Failure must be
    visible (an outcome, not an acceptance) and the FP64 guard must agree with
    the oracle.  Split BF16 (~16 bits) must converge and be certified."""
    dims, rmin = (32, 16, 16), 1e-4
    rho = synth.blobs(*dims, 1001)
    g = _gpu_grid(dims, rho, 3.0, rmin)
    b = np.random.default_rng(1).standard_normal(g.n_dof)
    z_ref, H = _oracle_vcycle(dims, rho, rmin, b)
    z = g.vcycle(torch.tensor(b, dtype=torch.float32, device=DEV), getattr(tg, prec)).cpu().numpy()
    tol = 0.05 if prec == "BF16MFMA" else 2e-3
    assert np.abs(z - z_ref).max() <= tol * np.abs(z_ref).max()
    og = mesh.Grid(*dims)
    free = og.free_dofs()
    ff = og.edge_load()[free]
    f = torch.tensor(g.edge_load(), device=DEV)
    u, res, hist = g.fgmres_solve(f, tg.solver_opts(prec=getattr(tg, prec)))
    eta = g.true_residual(f, u)
    if prec == "BF16X3MFMA":
        # inside FGMRES the split-BF16 cycle preconditions as well as the FP64
        # one (its first two sweeps run fused, reading the FP64 Krylov vector)
        _, r64, _ = g.fgmres_solve(f, tg.solver_opts(prec=tg.F64))
        assert res["iterations"] <= r64["iterations"] + 10
    if prec == "BF16X3MFMA" or res["outcome"] == "PROJ_CONVERGED":
        assert res["outcome"] == "PROJ_CONVERGED"
        assert eta <= 1e-6
        err, bnd = _solution_bound(H[0].K, ff, u.cpu().numpy()[free], eta)
        assert err <= bnd
    else:
        assert res["outcome"] in ("MAXIT", "BREAKDOWN") and res["proj_eta"] > 1e-6


def _valid_height(z, nz_nodes):
    return 1 <= z <= max(nz_nodes, 8)


def test_autotune_changes_only_the_decomposition():
    dims = (32, 16, 16)
    rho = _field("blob", dims, 21)
    g = _gpu_grid(dims, rho, 3.0, 1e-4)
    rng = np.random.default_rng(8)
    u64 = torch.tensor(rng.standard_normal(g.n_dof), device=DEV)
    u32 = u64.float()
    before = [g.apply_K(u64, tg.F64), g.apply_K(u32, tg.F32), g.vcycle(u64, tg.F64), g.vcycle(u32, tg.F32)]
    f = torch.tensor(g.edge_load(), device=DEV)
    u0, r0, _ = g.fgmres_solve(f, tg.solver_opts(prec=tg.F32))
    zc, us = g.autotune(tg.F32, force=True)
    assert _valid_height(zc[0], 17) and _valid_height(zc[1], 9)
    assert us[0] > 0 and us[1] > 0
    after = [g.apply_K(u64, tg.F64), g.apply_K(u32, tg.F32), g.vcycle(u64, tg.F64), g.vcycle(u32, tg.F32)]
    for a, b in zip(before, after):
        # every node sums its element contributions in one fixed order whatever the tiling
        assert torch.equal(a, b)
    u1, r1, _ = g.fgmres_solve(f, tg.solver_opts(prec=tg.F32))
    assert r1["iterations"] == r0["iterations"] and torch.equal(u0, u1)
    # a second call finds the cached choice and times nothing
    zc2, us2 = g.autotune(tg.F32)
    assert zc2 == zc and all(x == -1.0 for x in us2)


def test_autotuned_uneven_batch_equals_untuned():
    dims_list = [(32, 16, 16), (48, 24, 24), (16, 8, 8), (32, 16, 16)]
    rhos = [synth.blobs(*d, 40 + i, blob=4) for i, d in enumerate(dims_list)]
    floors = [1e-3, 1e-4, 1e-3, 1e-6]
    fs, res = [], []
    for tune in (False, True):
        grids = [tg.Grid(*d, max_restart=30, device=DEV) for d in dims_list]
        batch = tg.Batch(grids)
        batch.set_density([torch.tensor(r, device=DEV) for r in rhos], 3.0, floors)
        if tune:
            zc, us = batch.autotune(tg.F32, force=True)
            assert _valid_height(zc[0], 25) and us[0] > 0
        fs = [torch.tensor(g.edge_load(), device=DEV) for g in grids]
        res.append(batch.solve(fs, tg.solver_opts(prec=tg.F32)))
    (ua, ra), (ub, rb) = res
    for i in range(len(dims_list)):
        assert ra[i]["iterations"] == rb[i]["iterations"]
        assert torch.equal(ua[i], ub[i])


@pytest.mark.parametrize("prec", [tg.F64, tg.F32])
def test_graph_replay_equals_direct_launches(prec):
    """Captured FGMRES steps replay bitwise like direct launches, replay after
    replay, with eager work and synchronizations in between."""
    dims = (16, 8, 8)
    g = _gpu_grid(dims, synth.uniform(*dims, 0), 3.0, 1e-3)
    f = torch.tensor(g.edge_load(), device=DEV)
    u0, r0, h0 = g.fgmres_solve(f, tg.solver_opts(prec=prec, restart=7))
    for rep in range(3):
        u1, r1, h1 = g.fgmres_solve(f, tg.solver_opts(prec=prec, restart=7, graphs=True))
        assert r1 == r0 and torch.equal(u1, u0) and np.array_equal(h1, h0), rep
        # eager work between replays
        y = g.apply_K(u1, tg.F64)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()


def test_graph_replay_in_uneven_batch():
    dims_list = [(16, 8, 8), (24, 12, 12), (16, 8, 8)]
    rhos = [synth.uniform(*dims_list[0], 0), synth.blobs(*dims_list[1], 7), synth.uniform(*dims_list[2], 9)]
    grids = [tg.Grid(*d, max_restart=30, device=DEV) for d in dims_list]
    batch = tg.Batch(grids)
    rho_d = [torch.tensor(r, device=DEV) for r in rhos]
    fs = [torch.tensor(g.edge_load(), device=DEV) for g in grids]
    batch.set_density(rho_d, 3.0, [1e-3, 1e-4, 1e-2])
    ref_u, ref_r = batch.solve(fs, tg.solver_opts(prec=tg.F32))
    for rep in range(3):
        batch.set_density(rho_d, 3.0, [1e-3, 1e-4, 1e-2])
        us, res = batch.solve(fs, tg.solver_opts(prec=tg.F32, graphs=True))
        for a, b, ra, rb in zip(us, ref_u, res, ref_r):
            assert ra == rb and torch.equal(a, b), rep
