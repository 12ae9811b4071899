"""Device-side control of the batched Krylov loop (addition (2)): runs of
Arnoldi steps between host reads of the status, with the step kernels
skipping problems that stopped on the device, leave every result bitwise as
a read after every step would (solutions, iteration counts, outcomes,
histories), for both Gram-Schmidt forms, with and without graph replay, for
one grid and for an uneven batch whose problems stop at different steps.
The autotuner's per-grid-size tile heights are valid and change nothing
but the work decomposition.  The bottom of the V-cycle (one launch from a
level that fits one workgroup's LDS) starts at each problem's own level, so
a batch of grids with different bottom levels solves each problem bit for
bit as it is solved alone."""
import numpy as np
import pytest
import torch

from paper_2607_26382_amd import synth
from paper_2607_26382_amd import topoguard as tg
from paper_2607_26382_amd._lib import TopoguardError

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("cgs", [2, 3, 1])
@pytest.mark.parametrize("graphs", [False, True])
def test_sync_every_single_grid_bitwise(cgs, graphs):
    dims = (16, 8, 8)
    g = tg.Grid(*dims, max_restart=30, device=DEV)
    g.set_density(torch.tensor(synth.uniform(*dims, 0), device=DEV), 3.0, 1e-3)
    f = torch.tensor(g.edge_load(), device=DEV)
    ref = g.fgmres_solve(f, tg.solver_opts(restart=7, cgs_passes=cgs, sync_every=1))
    for se in (2, 3, 8, 64):
        for rep in range(2 if graphs else 1):
            u, res, hist = g.fgmres_solve(f, tg.solver_opts(restart=7, cgs_passes=cgs, sync_every=se,
                                                            graphs=graphs))
            assert res == ref[1] and torch.equal(u, ref[0]) and np.array_equal(hist, ref[2]), (se, rep)
            torch.cuda.synchronize()


@pytest.mark.parametrize("graphs", [False, True])
def test_sync_every_uneven_batch_bitwise(graphs):
    """Problems of four sizes and floors that stop at different steps (one at
    the cap), so runs end with some problems gated off mid-run."""
    cases = [((16, 8, 8), synth.uniform(16, 8, 8, 0), 1e-3), ((24, 12, 12), synth.blobs(24, 12, 12, 7), 1e-4),
             ((32, 16, 16), synth.blobs(32, 16, 16, 1001), 1e-9), ((16, 8, 8), synth.blobs(16, 8, 8, 3), 1e-2),
             ((48, 24, 24), synth.blobs(48, 24, 24, 4001), 1e-6)]
    grids = [tg.Grid(*d, max_restart=30, device=DEV) for d, _, _ in cases]
    batch = tg.Batch(grids)
    rhos = [torch.tensor(r, device=DEV) for _, r, _ in cases]
    floors = [fl for _, _, fl in cases]
    fs = [torch.tensor(g.edge_load(), device=DEV) for g in grids]
    out = {}
    for se in (1, 5, 16):
        for rep in range(2 if graphs else 1):
            batch.set_density(rhos, 3.0, floors)
            us, res = batch.solve(fs, tg.solver_opts(max_iters=60, sync_every=se, graphs=graphs))
            out[(se, rep)] = (us, res, [batch.history(i) for i in range(len(cases))])
    us0, res0, h0 = out[(1, 0)]
    its = [r["iterations"] for r in res0]
    assert len(set(its)) >= 2                         # stops spread over the runs
    for key, (us, res, h) in out.items():
        for i in range(len(cases)):
            assert res[i] == res0[i], (key, i)
            assert torch.equal(us[i], us0[i]), (key, i)
            assert np.array_equal(h[i], h0[i]), (key, i)


def test_sync_every_must_be_positive():
    g = tg.Grid(8, 4, 4, max_restart=30, device=DEV)
    g.set_density(torch.full((g.n_elem,), 0.5, dtype=torch.float64, device=DEV), 3.0, 1e-3)
    f = torch.tensor(g.edge_load(), device=DEV)
    with pytest.raises(TopoguardError, match="sync_every"):
        g.fgmres_solve(f, tg.solver_opts(sync_every=0))


def test_per_size_tile_heights():
    dims_list = [(32, 16, 16), (48, 24, 24), (16, 8, 8), (32, 16, 16), (96, 48, 48)]
    grids = [tg.Grid(*d, max_restart=30, device=DEV) for d in dims_list]
    batch = tg.Batch(grids)
    rhos = [torch.tensor(synth.blobs(*d, 40 + i, blob=4), device=DEV) for i, d in enumerate(dims_list)]
    batch.set_density(rhos, 3.0, [1e-3] * len(dims_list))
    fs = [torch.tensor(g.edge_load(), device=DEV) for g in grids]
    u0, r0 = batch.solve(fs, tg.solver_opts(prec=tg.F32))
    batch.autotune(tg.F32, force=True)
    zc = [batch.tile_heights(i) for i in range(len(dims_list))]
    print("per-size tile heights", {dims_list[i]: zc[i] for i in range(len(dims_list))}, flush=True)
    assert zc[0] == zc[3]                              # one choice per size
    for d, z, g in zip(dims_list, zc, grids):
        assert len(z) == g.n_levels
        for l, h in enumerate(z):
            assert 1 <= h <= d[2] // (1 << l) + 1
    batch.set_density(rhos, 3.0, [1e-3] * len(dims_list))
    u1, r1 = batch.solve(fs, tg.solver_opts(prec=tg.F32))
    for i in range(len(dims_list)):
        assert r1[i]["iterations"] == r0[i]["iterations"] and torch.equal(u1[i], u0[i])


@pytest.mark.parametrize("prec", [tg.F32, tg.F64])
def test_bottom_levels_per_problem(prec):
    """32x16x16 and 48x24x24 start the one-launch bottom at level 2 in FP32,
    96x48x48 at level 3 (level 2 does not fit); in FP64 the levels differ
    again.  Every problem of the batch equals its own single-grid solve."""
    cases = [((32, 16, 16), 1e-4), ((96, 48, 48), 1e-3), ((48, 24, 24), 1e-6)]
    rhos = [torch.tensor(synth.blobs(*d, 4100 + i), device=DEV) for i, (d, _) in enumerate(cases)]
    opts = tg.solver_opts(prec=prec, max_iters=40)
    grids = [tg.Grid(*d, max_restart=30, device=DEV) for d, _ in cases]
    batch = tg.Batch(grids)
    batch.set_density(rhos, 3.0, [fl for _, fl in cases])
    fs = [torch.tensor(g.edge_load(), device=DEV) for g in grids]
    us, res = batch.solve(fs, opts)
    for i, (d, fl) in enumerate(cases):
        g = tg.Grid(*d, max_restart=30, device=DEV)
        g.set_density(rhos[i], 3.0, fl)
        u1, r1, _ = g.fgmres_solve(fs[i], opts)
        print(f"bottom levels {d} prec={prec}: batch {res[i]['iterations']} its, alone {r1['iterations']}",
              flush=True)
        assert r1["iterations"] == res[i]["iterations"] and torch.equal(u1, us[i])
        assert res[i]["iterations"] > 5


def test_batch_policy_equals_single_grid_policy():
    """While only part of a batch runs (the ladder's later rungs) the z-tile
    heights are capped for parallelism; heights change only the work
    decomposition, so every problem's policy result in the batch equals its
    single-grid policy bit for bit (attempts, iterations, guard values,
    solution)."""
    dims = (32, 16, 16)
    n = 8
    rhos = [torch.tensor(synth.blobs(*dims, 1000 + i), device=DEV) for i in range(n)]
    grids = [tg.Grid(*dims, max_restart=100, device=DEV) for _ in range(n)]
    batch = tg.Batch(grids)
    fs = [torch.tensor(g.edge_load(), device=DEV) for g in grids]
    pol = tg.policy(rungs=[1e-9, 1e-6, 1e-4, 1e-3],
                    solve=tg.solver_opts(restart=30, max_iters=200, prec=tg.BF16X3MFMA))
    us, outs = batch.select_floor(rhos, fs, pol)
    # (every stop inside a batched solve shrinks the running set, which caps
    # the heights on this batch: 8 problems give fewer than 1024 tiles)
    print("batch policy attempts", [len(o["attempts"]) for o in outs], flush=True)
    for i in range(n):
        u1, o1 = grids[i].select_floor(rhos[i], fs[i], pol)
        assert o1["rung"] == outs[i]["rung"] and o1["attempts"] == outs[i]["attempts"], i
        assert torch.equal(u1, us[i]), i
