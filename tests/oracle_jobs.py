"""Oracle runs for the GPU parity tests at the benchmark's own grid, executed
in worker processes (test infrastructure: calls only oracle/ and the seeded
generators).  At 64x32x32 one hierarchy build takes ~10 s and one FGMRES
iteration ~0.1 s on one host core, so the probe and the solve at every rung
run side by side while the GPU side of the tests proceeds."""
import os

import numpy as np

TAU = 1e-6


def severe_task(args):
    """kind "probe": the 100-iteration probe (restart 100) at `floor` and one
    V-cycle of a seeded vector; kind "solve": FGMRES(30), cap 200, at
    `floor`, its recomputed residual and the solution (full length)."""
    kind, seed, floor = args
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    from oracle import fgmres as ofg
    from oracle import ke, mesh
    from oracle import multigrid as omg
    from oracle import operator as op
    from paper_2607_26382_amd import synth

    dims, rho = synth.severe(seed)
    og = mesh.Grid(*dims)
    free = og.free_dofs()
    f = og.edge_load()[free]
    H = omg.build_hierarchy(og, op.young(rho, 3.0, floor), ke.ke())
    A = lambda v: H[0].K @ v
    M = lambda v: omg.vcycle(H, v)
    if kind == "probe":
        r = ofg.fgmres(A, M, f, 100, 100, TAU)
        b = np.random.default_rng(seed).standard_normal(og.n_dof)
        z = np.zeros(og.n_dof)
        z[free] = omg.vcycle(H, b[free])
        return dict(hist=r.hist, iters=r.iters, outcome=r.outcome, b=b, z=z, levels=len(H))
    r = ofg.fgmres(A, M, f, 30, 200, TAU)
    x = np.zeros(og.n_dof)
    x[free] = r.x
    return dict(hist=r.hist, iters=r.iters, outcome=r.outcome, proj=r.proj_eta,
                eta=op.relative_residual(H[0].K, f, r.x), x=x)


def grid_task(args):
    """FGMRES(restart), cap 200, on one (grid, density, floor): the history,
    iterations, outcome and solution, for per-problem checks in a batch."""
    dims, rho, floor, restart = args
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    from oracle import fgmres as ofg
    from oracle import ke, mesh
    from oracle import multigrid as omg
    from oracle import operator as op

    og = mesh.Grid(*dims)
    free = og.free_dofs()
    f = og.edge_load()[free]
    H = omg.build_hierarchy(og, op.young(rho, 3.0, floor), ke.ke())
    r = ofg.fgmres(lambda v: H[0].K @ v, lambda v: omg.vcycle(H, v), f, restart, 200, TAU)
    x = np.zeros(og.n_dof)
    x[free] = r.x
    return dict(hist=r.hist, iters=r.iters, outcome=r.outcome, x=x)
