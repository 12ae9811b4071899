"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and its host-only calls (grid setup, Ke, load, workspace sizing)
agree with the oracle.  No compute call runs here."""
import ctypes as C
import os

import numpy as np
import pytest

from oracle import ke as oke
from oracle import mesh
from oracle import multigrid as omg

L = pytest.importorskip("paper_2607_26382_amd._lib")

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH),
                                reason="libtopoguard.so not built (run __graft_entry__.build())")


def test_exports_every_header_symbol():
    lib = L.lib()
    syms = L.header_symbols()
    assert len(syms) >= 25
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    assert set(L.PROTOTYPES) == set(syms)


def _grid(dims, mg=None):
    h = C.c_void_p()
    L.check(L.lib().tg_setup_grid(*dims, 1.0, 0.3, C.byref(mg) if mg else None, C.byref(h)))
    return h


@pytest.mark.parametrize("dims", [(16, 8, 8), (64, 32, 32), (48, 24, 24), (96, 48, 48),
                                  (256, 128, 128), (32, 16, 16), (17, 9, 7)])
def test_grid_info_matches_oracle(dims):
    h = _grid(dims)
    info = L.GridInfo()
    L.check(L.lib().tg_get_grid_info(h, C.byref(info)))
    levels = omg.level_dims(*dims)
    assert info.n_levels == len(levels)
    assert [tuple(info.level_dims[l]) for l in range(info.n_levels)] == levels
    nx, ny, nz = dims
    assert info.n_dof == 3 * (nx + 1) * (ny + 1) * (nz + 1)
    assert info.n_free == 3 * nx * (ny + 1) * (nz + 1)
    L.lib().tg_destroy(h)


def test_ke_and_load_match_oracle():
    h = _grid((12, 6, 4))
    ke = np.zeros(576)
    L.check(L.lib().tg_get_ke(h, ke.ctypes.data_as(C.POINTER(C.c_double))))
    assert np.max(np.abs(ke.reshape(24, 24) - oke.ke())) < 2e-16 * 4
    f = np.zeros(3 * 13 * 7 * 5)
    L.check(L.lib().tg_edge_load(h, f.ctypes.data_as(C.POINTER(C.c_double))))
    assert np.array_equal(f, mesh.Grid(12, 6, 4).edge_load())
    L.lib().tg_destroy(h)


def test_invalid_arguments_are_errors():
    lib = L.lib()
    h = C.c_void_p()
    assert lib.tg_setup_grid(0, 4, 4, 1.0, 0.3, None, C.byref(h)) == L.TG_EINVAL
    assert b"dimensions" in lib.tg_last_error()
    assert lib.tg_setup_grid(4, 4, 4, 1.0, 0.5, None, C.byref(h)) == L.TG_EINVAL
    mg = L.MgOpts(0, 300, 2.5, 2, 2)
    assert lib.tg_setup_grid(4, 4, 4, 1.0, 0.3, C.byref(mg), C.byref(h)) == L.TG_EINVAL
    h = _grid((8, 4, 4))
    nb = C.c_size_t()
    assert lib.tg_workspace_bytes(h, 0, C.byref(nb)) == L.TG_EINVAL
    L.check(lib.tg_workspace_bytes(h, 30, C.byref(nb)))
    assert nb.value > 0
    # calls that need a bound workspace refuse without one (no device touched)
    assert lib.tg_set_density(h, None, 3.0, 1e-3, None) == L.TG_ESTATE
    assert lib.tg_apply_K(h, None, None, 0, None) == L.TG_ESTATE
    lib.tg_destroy(h)


def test_workspace_accounting_grows_with_restart():
    h = _grid((64, 32, 32))
    a, b = C.c_size_t(), C.c_size_t()
    L.check(L.lib().tg_workspace_bytes(h, 30, C.byref(a)))
    L.check(L.lib().tg_workspace_bytes(h, 100, C.byref(b)))
    # two FP64 Krylov bases: 2 * 70 extra vectors of 3 * 70785 doubles (padded
    # to whole 2048-value reduction chunks), plus the (m+1) x m Hessenberg and
    # Givens scalars
    per_vec = ((3 * 33 * 33 * 65 + 2047) // 2048) * 2048 * 8
    small = 8 * (101 * 100 - 31 * 30 + 4 * 70)
    assert abs((b.value - a.value) - 140 * per_vec - small) < 4096
    L.lib().tg_destroy(h)


def test_default_structs():
    o = L.SolverOpts()
    L.lib().tg_default_solver_opts(C.byref(o))
    assert (o.restart, o.max_iters, o.tol, o.cgs_passes) == (30, 200, 1e-6, 2)
    m = L.MgOpts()
    L.lib().tg_default_mg_opts(C.byref(m))
    assert (m.max_coarse_dof, m.omega, m.nu_pre, m.nu_post) == (300, 0.6, 2, 2)
    p = L.Policy()
    L.lib().tg_default_policy(C.byref(p))
    assert p.n_rungs == 4 and list(p.rungs[:4]) == [1e-9, 1e-6, 1e-4, 1e-3]
    assert (p.t_high, p.t_plateau, p.t_ratio, p.probe_iters) == (1e-2, 1e-4, 0.6, 100)


def test_default_topopt_struct():
    # Tab. trajectory-settings; the nested policy sits at the end of the struct,
    # so a layout mismatch would garble it
    o = L.TopoptOpts()
    L.lib().tg_default_topopt(C.byref(o))
    assert (o.max_iters, o.min_iters, o.tol, o.volfrac, o.r_min, o.eta) == (40, 20, 0.01, 0.30, 1.5, 0.5)
    assert o.n_stages == 2 and o.mode == L.TG_LOOP_GUARDED
    assert [(s.first_iter, s.p, s.beta, s.move) for s in o.stages[:2]] == [(1, 1.5, 1.0, 0.20), (16, 3.5, 4.0, 0.15)]
    assert o.policy.n_rungs == 3 and list(o.policy.rungs[:3]) == [1e-12, 1e-3, 1e-2]
    assert (o.policy.t_high, o.policy.probe_iters, o.policy.solve.restart) == (1e-2, 100, 30)
    assert C.sizeof(L.TopoptRecord) == 96


def test_adaptive_workspace_sizing():
    """Host-only: the adaptive path's workspace holds the outer basis (2m + 1
    vectors), the inner basis (2q + 1), four work vectors, two float vectors
    and a Hessenberg of the inner iteration; restart and inner steps outside
    [0, TG_AD_MAX_RESTART] are errors."""
    h = _grid((16, 8, 8))
    info = L.GridInfo()
    L.check(L.lib().tg_get_grid_info(h, C.byref(info)))
    vb = ((info.n_dof + 31) // 32 * 32) * 8
    nb = C.c_size_t()

    def size(m, q):
        L.check(L.lib().tg_adaptive_workspace_bytes(h, m, q, C.byref(nb)))
        return nb.value

    base = size(0, 0)
    assert base >= 4 * vb + 2 * info.n_dof * 4
    assert size(30, 0) - base == 61 * vb
    assert size(0, 20) - base >= 41 * vb + 21 * 20 * 8
    assert size(L.TG_AD_MAX_RESTART, 20) > size(30, 20)
    for m, q in ((L.TG_AD_MAX_RESTART + 1, 20), (30, L.TG_AD_MAX_RESTART + 1), (-1, 0), (0, -1)):
        assert L.lib().tg_adaptive_workspace_bytes(h, m, q, C.byref(nb)) == L.TG_EINVAL
    L.lib().tg_destroy(h)
