"""Thin torch-facing binding of libtopoguard (argument marshalling only).

Device memory comes from torch (workspaces and vectors are torch tensors on the
current HIP device); every computation runs in the library's kernels.  Names
follow the C ABI: setup_grid, set_density, apply_K, vcycle, fgmres_solve,
true_residual, probe_features, select_floor.
"""
import ctypes as C

import numpy as np
import torch

from . import _lib as L
from ._lib import check, lib

F64, F32, BF16MFMA, BF16X3MFMA = L.TG_F64, L.TG_F32, L.TG_BF16MFMA, L.TG_BF16X3MFMA
OUTCOMES = {0: "PROJ_CONVERGED", 1: "MAXIT", 2: "BREAKDOWN", 3: "NONFINITE"}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _alloc_ws(nbytes, device):
    ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws, ws.data_ptr() + off


def mg_opts(max_levels=0, max_coarse_dof=300, omega=0.6, nu_pre=2, nu_post=2):
    return L.MgOpts(max_levels, max_coarse_dof, omega, nu_pre, nu_post)


def solver_opts(restart=30, max_iters=200, tol=1e-6, prec=F64, cgs_passes=2, breakdown=1e-14, graphs=False,
                sync_every=8):
    return L.SolverOpts(restart, max_iters, tol, prec, cgs_passes, breakdown, int(bool(graphs)), sync_every)


def policy(rungs=(1e-9, 1e-6, 1e-4, 1e-3), p=3.0, tau=1e-6, probe_iters=100, probe_restart=100,
           t_high=1e-2, t_plateau=1e-4, t_ratio=0.6, selector=L.TG_SELECT_RULE, fixed_rung=0,
           mlp=None, solve=None, want_features=False):
    pol = L.Policy()
    lib().tg_default_policy(C.byref(pol))
    pol.n_rungs = len(rungs)
    for i, r in enumerate(rungs):
        pol.rungs[i] = r
    pol.p, pol.tau = p, tau
    pol.probe_iters, pol.probe_restart = probe_iters, probe_restart
    pol.t_high, pol.t_plateau, pol.t_ratio = t_high, t_plateau, t_ratio
    pol.selector, pol.fixed_rung = selector, fixed_rung
    pol.mlp = mlp.handle if mlp is not None else None
    pol.solve = solve if solve is not None else solver_opts()
    pol.want_features = int(bool(want_features))
    return pol


def stack_opts(inner_steps=20, coarse_steps=10, nu_pre=2, nu_post=2, power_iters=10, lo=0.1, hi=1.1, theta=0.95):
    return L.StackOpts(inner_steps, coarse_steps, nu_pre, nu_post, power_iters, lo, hi, theta)


def stack_log_dict(g):
    return dict(alpha=g.alpha, ratio=g.ratio, coarse_accepted=bool(g.coarse_accepted), fine_kept=bool(g.fine_kept))


def result_dict(r):
    return dict(iterations=r.iterations, outcome=OUTCOMES.get(r.outcome, r.outcome),
                proj_eta=r.proj_eta, true_eta=r.true_eta)


def policy_dict(r):
    return dict(rung=r.rung, floor=r.floor, k0=r.k0, r50=r.r50, r100=r.r100,
                probe_iters=r.probe_iters, iters_probe=r.iters_probe,
                iters_selected=r.iters_selected, iters_rejected=r.iters_rejected,
                features=list(r.features),
                attempts=[dict(rung=a.rung, floor=a.floor, iterations=a.iterations,
                               outcome=OUTCOMES.get(a.outcome, a.outcome), proj_eta=a.proj_eta,
                               true_eta=a.true_eta, accepted=bool(a.accepted))
                          for a in r.attempts[:r.n_attempts]])


class Grid:
    """One structured cantilever grid with its device workspace (tg_grid)."""

    def __init__(self, nx, ny, nz, E0=1.0, nu=0.3, mg=None, max_restart=30, device=None):
        self.handle = C.c_void_p()
        check(lib().tg_setup_grid(nx, ny, nz, E0, nu, C.byref(mg) if mg is not None else None,
                                  C.byref(self.handle)))
        info = L.GridInfo()
        check(lib().tg_get_grid_info(self.handle, C.byref(info)))
        self.info = info
        self.nx, self.ny, self.nz = nx, ny, nz
        self.n_elem, self.n_nodes, self.n_dof = info.n_elem, info.n_nodes, info.n_dof
        self.n_levels = info.n_levels
        self.level_dims = [tuple(info.level_dims[l]) for l in range(info.n_levels)]
        self.max_restart = max_restart
        self.device = device
        self.ws = None
        if device is not None:
            self.bind(device, max_restart)

    def bind(self, device="cuda", max_restart=None):
        if max_restart is not None:
            self.max_restart = max_restart
        nb = C.c_size_t()
        check(lib().tg_workspace_bytes(self.handle, self.max_restart, C.byref(nb)))
        self.ws, ptr = _alloc_ws(nb.value, device)
        self.device = device
        check(lib().tg_bind_workspace(self.handle, C.c_void_p(ptr), nb.value, self.max_restart))
        self.ws_bytes = nb.value
        return self

    def __del__(self):
        try:
            if self.handle:
                lib().tg_destroy(self.handle)
                self.handle = C.c_void_p()
        except Exception:
            pass

    # ---- host-side facts
    def ke(self):
        out = np.zeros(576)
        check(lib().tg_get_ke(self.handle, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(24, 24)

    def edge_load(self):
        f = np.zeros(self.n_dof)
        check(lib().tg_edge_load(self.handle, f.ctypes.data_as(C.POINTER(C.c_double))))
        return f

    # ---- device calls
    def set_density(self, rho, p, rho_min):
        assert rho.dtype == torch.float64 and rho.is_cuda and rho.numel() == self.n_elem
        self._rho = rho.contiguous()
        check(lib().tg_set_density(self.handle, _ptr(self._rho), float(p), float(rho_min), _stream()))

    def apply_K(self, u, prec=F64):
        dt = torch.float64 if prec == F64 else torch.float32
        assert u.dtype == dt and u.numel() == self.n_dof
        y = torch.empty_like(u)
        check(lib().tg_apply_K(self.handle, _ptr(u), _ptr(y), prec, _stream()))
        return y

    def vcycle(self, r, prec=F64):
        dt = torch.float64 if prec == F64 else torch.float32
        assert r.dtype == dt and r.numel() == self.n_dof
        z = torch.empty_like(r)
        check(lib().tg_vcycle(self.handle, _ptr(r), _ptr(z), prec, _stream()))
        return z

    def fgmres_solve(self, f, opts=None, want_hist=True):
        opts = opts or solver_opts()
        u = torch.empty_like(f)
        res = L.SolveResult()
        hist = np.zeros(4096)
        check(lib().tg_fgmres_solve(self.handle, _ptr(f), _ptr(u), C.byref(opts), C.byref(res),
                                    hist.ctypes.data_as(C.POINTER(C.c_double)) if want_hist else None,
                                    _stream()))
        return u, result_dict(res), hist[:res.iterations + 1].copy()

    def true_residual(self, f, u):
        eta = C.c_double()
        check(lib().tg_true_residual(self.handle, _ptr(f), _ptr(u), C.byref(eta), _stream()))
        return eta.value

    def probe_features(self, f, iters=100, restart=100, prec=F64):
        o = solver_opts(restart=restart, max_iters=iters, prec=prec)
        r50, r100, ks = C.c_double(), C.c_double(), C.c_int()
        check(lib().tg_probe_features(self.handle, _ptr(f), C.byref(o), iters, C.byref(r50),
                                      C.byref(r100), C.byref(ks), _stream()))
        return r50.value, r100.value, ks.value

    def probe_checkpoints(self, f, iters=100, restart=100, every=10, prec=F64):
        """The probe with true-residual checkpoints: (list of (k, projected,
        true), k_stop)."""
        o = solver_opts(restart=restart, max_iters=iters, prec=prec)
        cap = iters // max(int(every), 1) + 1
        ks, pj, tr = (C.c_int * cap)(), (C.c_double * cap)(), (C.c_double * cap)()
        n, kst = C.c_int(), C.c_int()
        check(lib().tg_probe_checkpoints(self.handle, _ptr(f), C.byref(o), iters, every, cap, ks, pj, tr,
                                         C.byref(n), C.byref(kst), _stream()))
        return [(ks[i], pj[i], tr[i]) for i in range(n.value)], kst.value

    def adaptive_precondition(self, v, prec=F64, inner_steps=20):
        """(z, accepted): one V-cycle plus the fine-level correction, kept if
        it lowers the residual norm (v, z device FP64)."""
        assert v.dtype == torch.float64 and v.is_cuda and v.numel() == self.n_dof
        nb = C.c_size_t()
        check(lib().tg_adaptive_workspace_bytes(self.handle, 0, int(inner_steps), C.byref(nb)))
        ws, wptr = _alloc_ws(nb.value, self.device)
        z = torch.empty_like(v)
        acc = C.c_int()
        check(lib().tg_adaptive_precondition(self.handle, _ptr(v), _ptr(z), prec, int(inner_steps),
                                             C.c_void_p(wptr), nb.value, C.byref(acc), _stream()))
        del ws
        return z, bool(acc.value)

    def adaptive_solve(self, f, opts=None, inner_steps=20):
        """(u, result dict, history, accepted flags per preconditioner
        application): FGMRES with the adaptive preconditioner."""
        opts = opts or solver_opts()
        nb = C.c_size_t()
        check(lib().tg_adaptive_workspace_bytes(self.handle, opts.restart, int(inner_steps), C.byref(nb)))
        ws, wptr = _alloc_ws(nb.value, self.device)
        u = torch.empty_like(f)
        res = L.SolveResult()
        hist = np.zeros(opts.max_iters + 1)
        acc = (C.c_int * (opts.max_iters + 1))()
        na = C.c_int()
        check(lib().tg_adaptive_solve(self.handle, _ptr(f), _ptr(u), C.byref(opts), int(inner_steps),
                                      C.c_void_p(wptr), nb.value, C.byref(res),
                                      hist.ctypes.data_as(C.POINTER(C.c_double)), acc, C.byref(na), _stream()))
        del ws
        n = min(na.value, opts.max_iters + 1)
        return u, result_dict(res), hist[:res.iterations + 1].copy(), [bool(acc[i]) for i in range(n)]

    def adaptive_checkpoints(self, f, opts=None, inner_steps=20, every=10):
        """(u, result dict, [(k, projected, true)]): the adaptive solve with a
        recomputed residual of the iterate every `every` iterations."""
        opts = opts or solver_opts()
        nb = C.c_size_t()
        check(lib().tg_adaptive_workspace_bytes(self.handle, opts.restart, int(inner_steps), C.byref(nb)))
        ws, wptr = _alloc_ws(nb.value, self.device)
        u = torch.empty_like(f)
        res = L.SolveResult()
        cap = opts.max_iters // max(int(every), 1) + 1
        ks, pj, tr, n = (C.c_int * cap)(), (C.c_double * cap)(), (C.c_double * cap)(), C.c_int()
        check(lib().tg_adaptive_checkpoints(self.handle, _ptr(f), _ptr(u), C.byref(opts), int(inner_steps),
                                            int(every), cap, C.c_void_p(wptr), nb.value, C.byref(res), ks, pj, tr,
                                            C.byref(n), _stream()))
        del ws
        return u, result_dict(res), [(ks[i], pj[i], tr[i]) for i in range(n.value)]

    def _stack_ws(self, restart, so):
        nb = C.c_size_t()
        check(lib().tg_stack_workspace_bytes(self.handle, int(restart), C.byref(so), C.byref(nb)))
        ws, wptr = _alloc_ws(nb.value, self.device)
        return ws, C.c_void_p(wptr), nb.value

    def stack_lambdas(self, so=None):
        """lambda~ of every level above the coarsest (power estimates of the
        largest eigenvalue of D^-1 K, the Chebyshev intervals' scale)."""
        so = so or stack_opts()
        ws, wptr, nb = self._stack_ws(0, so)
        out = (C.c_double * 8)()
        check(lib().tg_stack_lambdas(self.handle, C.byref(so), wptr, nb, out, _stream()))
        del ws
        return [out[i] for i in range(self.n_levels - 1)]

    def stack_precondition(self, v, so=None, lams=None):
        """(z, log dict): one application of the full adaptive stack (v, z
        device FP64); lams: lambda~ per level, or None to estimate them."""
        assert v.dtype == torch.float64 and v.is_cuda and v.numel() == self.n_dof
        so = so or stack_opts()
        ws, wptr, nb = self._stack_ws(0, so)
        z = torch.empty_like(v)
        lg = L.StackLog()
        lam = None if lams is None else (C.c_double * len(lams))(*[float(x) for x in lams])
        check(lib().tg_stack_precondition(self.handle, _ptr(v), _ptr(z), C.byref(so), lam, wptr, nb, C.byref(lg),
                                          _stream()))
        del ws
        return z, stack_log_dict(lg)

    def stack_solve(self, f, opts=None, so=None):
        """(u, result dict, history, per-application logs, lambda~): FGMRES
        preconditioned by the full adaptive stack."""
        opts = opts or solver_opts()
        so = so or stack_opts()
        ws, wptr, nb = self._stack_ws(opts.restart, so)
        u = torch.empty_like(f)
        res = L.SolveResult()
        hist = np.zeros(opts.max_iters + 1)
        logs = (L.StackLog * (opts.max_iters + 1))()
        na = C.c_int()
        lams = (C.c_double * 8)()
        check(lib().tg_stack_solve(self.handle, _ptr(f), _ptr(u), C.byref(opts), C.byref(so), wptr, nb,
                                   C.byref(res), hist.ctypes.data_as(C.POINTER(C.c_double)), logs, C.byref(na),
                                   lams, _stream()))
        del ws
        n = min(na.value, opts.max_iters + 1)
        nl = self.n_levels - 1
        return (u, result_dict(res), hist[:res.iterations + 1].copy(), [stack_log_dict(logs[i]) for i in range(n)],
                [lams[i] for i in range(nl)])

    def stack_select_floor(self, rho, f, pol, so=None):
        """(u, policy dict): Alg. floor_policy with the full adaptive stack
        preconditioning the probe and every rung's solve."""
        so = so or stack_opts()
        ws, wptr, nb = self._stack_ws(max(pol.probe_restart, pol.solve.restart), so)
        u = torch.empty_like(f)
        out = L.PolicyResult()
        check(lib().tg_stack_select_floor(self.handle, _ptr(rho), _ptr(f), C.byref(pol), C.byref(so), wptr, nb,
                                          _ptr(u), C.byref(out), _stream()))
        del ws
        return u, policy_dict(out)

    def density_features(self, rho, p=3.0, rho0=1e-9):
        """Six density statistics of rho (device FP64) at probe floor rho0."""
        out = (C.c_double * 6)()
        check(lib().tg_density_features(self.handle, _ptr(rho), float(p), float(rho0), out, _stream()))
        return list(out)

    def compliance_sensitivity(self, u, f=None, rho=None, p=3.0, rho_min=1e-3, want_energy=False):
        """dict(compliance=f^T u or None, dc=sensitivities or None, energy=u_e^T K_e u_e or None)
        for a displacement u (device FP64).  dc needs rho, the compliance needs f."""
        assert u.dtype == torch.float64 and u.is_cuda and u.numel() == self.n_dof
        dc = torch.empty(self.n_elem, dtype=torch.float64, device=u.device) if rho is not None else None
        en = torch.empty(self.n_elem, dtype=torch.float64, device=u.device) if want_energy else None
        c = C.c_double()
        check(lib().tg_compliance_sensitivity(
            self.handle, _ptr(rho) if rho is not None else None, float(p), float(rho_min),
            _ptr(f) if f is not None else None, _ptr(u), _ptr(en) if en is not None else None,
            _ptr(dc) if dc is not None else None, C.byref(c) if f is not None else None, _stream()))
        return {"compliance": c.value if f is not None else None, "dc": dc, "energy": en}

    def gradient_change(self, rho, dc0, dc1, solid_min=0.5):
        """Relative l2 change and Pearson r of dc1 against dc0 over rho >= solid_min."""
        out = L.GradientChange()
        check(lib().tg_gradient_change(self.handle, _ptr(rho), float(solid_min), _ptr(dc0), _ptr(dc1),
                                       C.byref(out), _stream()))
        return {"n_solid": out.n_solid, "rel_l2": out.rel_l2, "pearson": out.pearson,
                "norm0": out.norm0, "norm1": out.norm1}

    def extreme_eigenvalues(self, prec=F64, max_iters=300, tol=1e-8):
        """dict(lambda_min, lambda_max, kappa, resid_min, iters_min, iters_max,
        converged) of the operator of the last set_density."""
        nb = C.c_size_t()
        check(lib().tg_spectrum_workspace_bytes(self.handle, C.byref(nb)))
        ws, wptr = _alloc_ws(nb.value, self.device)
        out = L.SpectrumResult()
        check(lib().tg_extreme_eigenvalues(self.handle, prec, int(max_iters), float(tol), C.c_void_p(wptr),
                                           nb.value, C.byref(out), _stream()))
        del ws
        return {k: getattr(out, k) for k, _ in L.SpectrumResult._fields_}

    # ---- the optimizer around the solve
    def _efield(self, t):
        assert t.dtype == torch.float64 and t.is_cuda and t.numel() == self.n_elem
        return _ptr(t)

    def density_filter(self, x, r_min=1.5):
        y = torch.empty_like(x)
        check(lib().tg_density_filter(self.handle, self._efield(x), float(r_min), _ptr(y), _stream()))
        return y

    def density_filter_adjoint(self, a, b=None, r_min=1.5):
        y = torch.empty_like(a)
        check(lib().tg_density_filter_adjoint(self.handle, self._efield(a),
                                              self._efield(b) if b is not None else None, float(r_min),
                                              _ptr(y), _stream()))
        return y

    def filter_project(self, x, r_min=1.5, beta=1.0, eta=0.5):
        """(xt, xbar, dxbar) = (H x, project(H x), d project / d xt)."""
        xt, xb, dx = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
        check(lib().tg_filter_project(self.handle, self._efield(x), float(r_min), float(beta), float(eta),
                                      _ptr(xt), _ptr(xb), _ptr(dx), _stream()))
        return xt, xb, dx

    def oc_update(self, x, dc, dv, volfrac, move, r_min=1.5, beta=1.0, eta=0.5):
        xn = torch.empty_like(x)
        lam = C.c_double()
        check(lib().tg_oc_update(self.handle, self._efield(x), self._efield(dc), self._efield(dv), float(volfrac),
                                 float(move), float(r_min), float(beta), float(eta), _ptr(xn), C.byref(lam),
                                 _stream()))
        return xn, lam.value

    def topopt_run(self, x0, f, opts):
        """Runs the optimization loop from design x0 (copied); returns the
        final design and one dict per outer iteration."""
        nb = C.c_size_t()
        check(lib().tg_topopt_workspace_bytes(self.handle, C.byref(nb)))
        ws, wptr = _alloc_ws(nb.value, x0.device)
        x = x0.clone()
        rec = (L.TopoptRecord * opts.max_iters)()
        n = C.c_int()
        check(lib().tg_topopt_run(self.handle, _ptr(f), C.byref(opts), C.c_void_p(wptr), nb.value,
                                  self._efield(x), rec, C.byref(n), _stream()))
        del ws
        keys = [k for k, _ in L.TopoptRecord._fields_]
        return x, [{k: getattr(rec[i], k) for k in keys} for i in range(n.value)]

    def autotune(self, prec=F32, force=False):
        zc, us = (C.c_int * 8)(), (C.c_double * 8)()
        check(lib().tg_autotune(self.handle, prec, int(force), zc, us, _stream()))
        return list(zc)[:self.n_levels], list(us)[:self.n_levels]

    def select_floor(self, rho, f, pol):
        u = torch.empty_like(f)
        out = L.PolicyResult()
        check(lib().tg_select_floor(self.handle, _ptr(rho), _ptr(f), C.byref(pol), _ptr(u),
                                    C.byref(out), _stream()))
        return u, policy_dict(out)


def gradient_change_noalloc(rho, dc0, dc1, solid_min=0.5):
    """tg_gradient_change_noalloc: the comparison of Grid.gradient_change on
    n = rho.numel() elements, with no grid and no device allocation."""
    out = L.GradientChange()
    check(lib().tg_gradient_change_noalloc(rho.numel(), _ptr(rho), float(solid_min), _ptr(dc0), _ptr(dc1),
                                           C.byref(out), _stream()))
    return {"n_solid": out.n_solid, "rel_l2": out.rel_l2, "pearson": out.pearson,
            "norm0": out.norm0, "norm1": out.norm1}


class Batch:
    """Independent problems of possibly different grid sizes solved together."""

    def __init__(self, grids):
        self.grids = list(grids)
        arr = (C.c_void_p * len(self.grids))(*[g.handle.value for g in self.grids])
        self.handle = C.c_void_p()
        check(lib().tg_batch_create(len(self.grids), arr, C.byref(self.handle)))
        nb = C.c_size_t()
        check(lib().tg_batch_workspace_bytes(self.handle, C.byref(nb)))
        self.ws, ptr = _alloc_ws(nb.value, self.grids[0].device)
        check(lib().tg_batch_bind_workspace(self.handle, C.c_void_p(ptr), nb.value))

    def __del__(self):
        try:
            if self.handle:
                lib().tg_batch_destroy(self.handle)
                self.handle = C.c_void_p()
        except Exception:
            pass

    @staticmethod
    def _ptrs(ts):
        return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def set_density(self, rhos, p, rho_mins):
        self._rhos = [r.contiguous() for r in rhos]
        rm = (C.c_double * len(rhos))(*rho_mins)
        check(lib().tg_batch_set_density(self.handle, self._ptrs(self._rhos), float(p), rm, _stream()))

    def solve(self, fs, opts=None):
        opts = opts or solver_opts()
        us = [torch.empty_like(f) for f in fs]
        res = (L.SolveResult * len(fs))()
        check(lib().tg_batch_solve(self.handle, self._ptrs(fs), self._ptrs(us), C.byref(opts), res,
                                   _stream()))
        self._iters = [r.iterations for r in res]
        return us, [result_dict(r) for r in res]

    def tile_heights(self, i):
        """z-tile heights problem i uses at each of its levels."""
        z = (C.c_int * 8)()
        check(lib().tg_batch_tile_heights(self.handle, i, z))
        return [v for v in z if v > 0]

    def history(self, i):
        """Residual history of problem i of the last solve (iterations + 1 values)."""
        n = self._iters[i] + 1
        h = (C.c_double * n)()
        check(lib().tg_batch_history(self.handle, i, n, h, _stream()))
        return np.array(h[:])

    def autotune(self, prec=F32, force=False):
        zc, us = (C.c_int * 8)(), (C.c_double * 8)()
        check(lib().tg_batch_autotune(self.handle, prec, int(force), zc, us, _stream()))
        return list(zc), list(us)

    def select_floor(self, rhos, fs, pol):
        us = [torch.empty_like(f) for f in fs]
        out = (L.PolicyResult * len(fs))()
        check(lib().tg_batch_select_floor(self.handle, self._ptrs(rhos), self._ptrs(fs), C.byref(pol),
                                          self._ptrs(us), out, _stream()))
        return us, [policy_dict(r) for r in out]


SELECT_RULE, SELECT_MLP, SELECT_FIXED = L.TG_SELECT_RULE, L.TG_SELECT_MLP, L.TG_SELECT_FIXED
LOOP_GUARDED, LOOP_REUSE, LOOP_FIXED = L.TG_LOOP_GUARDED, L.TG_LOOP_REUSE, L.TG_LOOP_FIXED


def topopt_opts(mode=LOOP_GUARDED, max_iters=40, min_iters=20, tol=0.01, volfrac=0.30, r_min=1.5,
                stages=((1, 1.5, 1.0, 0.20), (16, 3.5, 4.0, 0.15)), fixed_floor=1e-3, policy=None):
    """Loop options (defaults: Tab. trajectory-settings); policy defaults to
    the library's with rungs 1e-12, 1e-3, 1e-2."""
    o = L.TopoptOpts()
    lib().tg_default_topopt(C.byref(o))
    o.mode, o.max_iters, o.min_iters, o.tol = mode, max_iters, min_iters, tol
    o.volfrac, o.r_min, o.fixed_floor = volfrac, r_min, fixed_floor
    o.n_stages = len(stages)
    for q, (it, p, beta, move) in enumerate(stages):
        o.stages[q].first_iter, o.stages[q].p, o.stages[q].beta, o.stages[q].move = it, p, beta, move
    if policy is not None:
        o.policy = policy
    return o
N_PARAMS = 4996


class MLP:
    """The 8-64-64-4 first-floor selector network (tg_mlp) with its device
    workspace; parameters in the C ABI order W1, b1, W2, b2, W3, b3."""

    def __init__(self, params=None, mean=None, std=None, max_batch=4096, device="cuda"):
        nb = C.c_size_t()
        check(lib().tg_mlp_workspace_bytes(max_batch, C.byref(nb)))
        self.ws, ptr = _alloc_ws(nb.value, device)
        self.handle = C.c_void_p()
        check(lib().tg_mlp_create(C.c_void_p(ptr), nb.value, max_batch, C.byref(self.handle)))
        self.device = device
        if params is not None:
            self.set_params(params, mean, std)

    def __del__(self):
        try:
            if self.handle:
                lib().tg_mlp_destroy(self.handle)
                self.handle = C.c_void_p()
        except Exception:
            pass

    @staticmethod
    def flatten(params):
        return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params]).astype(np.float32)

    @staticmethod
    def unflatten(flat):
        flat = np.asarray(flat, dtype=np.float64)
        shapes = [(64, 8), (64,), (64, 64), (64,), (4, 64), (4,)]
        out, o = [], 0
        for sh in shapes:
            n = int(np.prod(sh))
            out.append(flat[o:o + n].reshape(sh))
            o += n
        return out

    def set_params(self, params, mean=None, std=None):
        flat = self.flatten(params) if isinstance(params, (list, tuple)) else params
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == N_PARAMS
        fp = C.POINTER(C.c_float)
        mu = None if mean is None else np.ascontiguousarray(mean, dtype=np.float32)
        sd = None if std is None else np.ascontiguousarray(std, dtype=np.float32)
        check(lib().tg_mlp_set_params(self.handle, flat.ctypes.data_as(fp),
                                      mu.ctypes.data_as(fp) if mu is not None else None,
                                      sd.ctypes.data_as(fp) if sd is not None else None, _stream()))

    def get_params(self):
        out = np.zeros(N_PARAMS, dtype=np.float32)
        check(lib().tg_mlp_get_params(self.handle, out.ctypes.data_as(C.POINTER(C.c_float)), _stream()))
        return out

    def forward(self, x):
        """x: (B, 8) raw features (device float32) -> (B, 4) logits."""
        x = x.contiguous()
        out = torch.empty((x.shape[0], 4), dtype=torch.float32, device=x.device)
        check(lib().tg_mlp_forward(self.handle, _ptr(x), x.shape[0], _ptr(out), _stream()))
        return out

    def train_step(self, x, y, lr=1e-3, want_grads=False):
        """One Adam step on (x (B,8) float32, y (B,) int32), both on the device."""
        x, y = x.contiguous(), y.contiguous()
        loss = C.c_float()
        g = torch.empty(N_PARAMS, dtype=torch.float32, device=x.device) if want_grads else None
        check(lib().tg_mlp_train_step(self.handle, _ptr(x), _ptr(y), x.shape[0], float(lr), C.byref(loss),
                                      _ptr(g) if g is not None else None, _stream()))
        return (loss.value, g) if want_grads else loss.value


# ---- kernel-class timer (instrumentation) ----------------------------------
def kernel_timer_enable(mask=(1 << L.TG_KT_COUNT) - 1):
    check(lib().tg_timer_enable(int(mask)))


def kernel_timer_reset():
    check(lib().tg_timer_reset())


def kernel_timer_read():
    """{class name: dict(kind, count, ms, bytes, avg_us, gbs)} (harvests events)."""
    out = {}
    for k in range(L.TG_KT_COUNT):
        ms, n, by = C.c_double(), C.c_longlong(), C.c_double()
        check(lib().tg_timer_read(k, C.byref(ms), C.byref(n), C.byref(by)))
        name = lib().tg_timer_name(k).decode()
        avg = 1e3 * ms.value / n.value if n.value else 0.0
        gbs = by.value / (ms.value * 1e-3) / 1e9 if ms.value > 0 else 0.0
        out[name] = dict(kind=k, count=n.value, ms=ms.value, bytes=by.value, avg_us=avg, gbs=gbs)
    return out


def dominant_kernel(timers):
    """The byte-accounted class with the largest total time."""
    cands = [(v["ms"], k) for k, v in timers.items() if v["bytes"] > 0 and v["count"]]
    return max(cands)[1] if cands else None


def roofline_from_timers(timers, hbm_peak_gbs, traffic=None):
    k = dominant_kernel(timers)
    if k is None:
        return None
    v = timers[k]
    achieved = v["gbs"]
    return {"kernel": k, "bound": "hbm", "achieved": achieved, "peak": hbm_peak_gbs, "unit": "GB/s",
            "frac": achieved / hbm_peak_gbs, "traffic": traffic,
            "avg_launch_us": v["avg_us"], "launches": v["count"],
            "alg_bytes_per_launch": v["bytes"] / v["count"]}
