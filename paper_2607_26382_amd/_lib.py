"""ctypes view of libtopoguard.so (the C ABI declared in include/topoguard.h).

Loading fails loudly if the library has not been built: there is no fallback.
"""
import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtopoguard.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "topoguard.h")

TG_OK, TG_EINVAL, TG_EHIP, TG_EWORKSPACE, TG_ESTATE, TG_ENUMERIC = 0, -1, -2, -3, -4, -5
TG_F64, TG_F32, TG_BF16MFMA, TG_BF16X3MFMA = 0, 1, 2, 3
TG_PROJ_CONVERGED, TG_MAXIT, TG_BREAKDOWN, TG_NONFINITE = 0, 1, 2, 3
TG_SELECT_RULE, TG_SELECT_MLP, TG_SELECT_FIXED = 0, 1, 2
TG_MAX_RUNGS = 8
TG_LOOP_GUARDED, TG_LOOP_REUSE, TG_LOOP_FIXED = 0, 1, 2


class MgOpts(C.Structure):
    _fields_ = [("max_levels", C.c_int), ("max_coarse_dof", C.c_int), ("omega", C.c_double),
                ("nu_pre", C.c_int), ("nu_post", C.c_int)]


class SolverOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_iters", C.c_int), ("tol", C.c_double),
                ("prec", C.c_int), ("cgs_passes", C.c_int), ("breakdown", C.c_double),
                ("graphs", C.c_int), ("sync_every", C.c_int)]


class SolveResult(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outcome", C.c_int), ("proj_eta", C.c_double),
                ("true_eta", C.c_double)]


class GridInfo(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("n_elem", C.c_int64), ("n_nodes", C.c_int64), ("n_dof", C.c_int64),
                ("n_free", C.c_int64), ("n_levels", C.c_int),
                ("level_dims", (C.c_int * 3) * 8), ("coarse_free_dof", C.c_int)]


class Policy(C.Structure):
    _fields_ = [("n_rungs", C.c_int), ("rungs", C.c_double * TG_MAX_RUNGS), ("p", C.c_double),
                ("tau", C.c_double), ("probe_iters", C.c_int), ("probe_restart", C.c_int),
                ("t_high", C.c_double), ("t_plateau", C.c_double), ("t_ratio", C.c_double),
                ("selector", C.c_int), ("fixed_rung", C.c_int), ("mlp", C.c_void_p),
                ("solve", SolverOpts), ("want_features", C.c_int)]


class StackOpts(C.Structure):
    _fields_ = [("inner_steps", C.c_int), ("coarse_steps", C.c_int), ("nu_pre", C.c_int), ("nu_post", C.c_int),
                ("power_iters", C.c_int), ("lo", C.c_double), ("hi", C.c_double), ("theta", C.c_double)]


class StackLog(C.Structure):
    _fields_ = [("alpha", C.c_double), ("ratio", C.c_double), ("coarse_accepted", C.c_int),
                ("fine_kept", C.c_int)]


class Attempt(C.Structure):
    _fields_ = [("rung", C.c_int), ("iterations", C.c_int), ("outcome", C.c_int),
                ("accepted", C.c_int), ("floor", C.c_double), ("proj_eta", C.c_double),
                ("true_eta", C.c_double)]


class GradientChange(C.Structure):
    _fields_ = [("n_solid", C.c_int64), ("rel_l2", C.c_double), ("pearson", C.c_double),
                ("norm0", C.c_double), ("norm1", C.c_double)]


class SpectrumResult(C.Structure):
    _fields_ = [("lambda_min", C.c_double), ("lambda_max", C.c_double), ("kappa", C.c_double),
                ("resid_min", C.c_double), ("iters_min", C.c_int), ("iters_max", C.c_int),
                ("converged", C.c_int)]


class Stage(C.Structure):
    _fields_ = [("first_iter", C.c_int), ("p", C.c_double), ("beta", C.c_double), ("move", C.c_double)]


class TopoptOpts(C.Structure):
    _fields_ = [("max_iters", C.c_int), ("min_iters", C.c_int), ("tol", C.c_double),
                ("volfrac", C.c_double), ("r_min", C.c_double), ("eta", C.c_double),
                ("n_stages", C.c_int), ("stages", Stage * 4), ("mode", C.c_int),
                ("fixed_floor", C.c_double), ("policy", Policy)]


class TopoptRecord(C.Structure):
    _fields_ = [("iter", C.c_int), ("p", C.c_double), ("beta", C.c_double), ("compliance", C.c_double),
                ("volume", C.c_double), ("change", C.c_double), ("rung", C.c_int), ("floor", C.c_double),
                ("probed", C.c_int), ("solve_iters", C.c_int), ("true_eta", C.c_double),
                ("accepted", C.c_int), ("ms", C.c_double)]


class PolicyResult(C.Structure):
    _fields_ = [("rung", C.c_int), ("floor", C.c_double), ("k0", C.c_int), ("r50", C.c_double),
                ("r100", C.c_double), ("probe_iters", C.c_int), ("n_attempts", C.c_int),
                ("attempts", Attempt * TG_MAX_RUNGS), ("iters_probe", C.c_int),
                ("iters_selected", C.c_int), ("iters_rejected", C.c_int),
                ("features", C.c_double * 8)]


_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_SZ = C.c_size_t

PROTOTYPES = {
    "tg_last_error": (C.c_char_p, []),
    "tg_default_mg_opts": (None, [C.POINTER(MgOpts)]),
    "tg_default_solver_opts": (None, [C.POINTER(SolverOpts)]),
    "tg_setup_grid": (_I, [_I, _I, _I, _D, _D, C.POINTER(MgOpts), C.POINTER(_P)]),
    "tg_destroy": (None, [_P]),
    "tg_get_grid_info": (_I, [_P, C.POINTER(GridInfo)]),
    "tg_get_ke": (_I, [_P, C.POINTER(_D)]),
    "tg_edge_load": (_I, [_P, C.POINTER(_D)]),
    "tg_workspace_bytes": (_I, [_P, _I, C.POINTER(_SZ)]),
    "tg_bind_workspace": (_I, [_P, _P, _SZ, _I]),
    "tg_set_density": (_I, [_P, _P, _D, _D, _P]),
    "tg_apply_K": (_I, [_P, _P, _P, _I, _P]),
    "tg_vcycle": (_I, [_P, _P, _P, _I, _P]),
    "tg_fgmres_solve": (_I, [_P, _P, _P, C.POINTER(SolverOpts), C.POINTER(SolveResult),
                             C.POINTER(_D), _P]),
    "tg_true_residual": (_I, [_P, _P, _P, C.POINTER(_D), _P]),
    "tg_probe_features": (_I, [_P, _P, C.POINTER(SolverOpts), _I, C.POINTER(_D), C.POINTER(_D),
                               C.POINTER(_I), _P]),
    "tg_probe_checkpoints": (_I, [_P, _P, C.POINTER(SolverOpts), _I, _I, _I, C.POINTER(_I), C.POINTER(_D),
                                  C.POINTER(_D), C.POINTER(_I), C.POINTER(_I), _P]),
    "tg_default_policy": (None, [C.POINTER(Policy)]),
    "tg_select_floor": (_I, [_P, _P, _P, C.POINTER(Policy), _P, C.POINTER(PolicyResult), _P]),
    "tg_batch_create": (_I, [_I, C.POINTER(_P), C.POINTER(_P)]),
    "tg_batch_destroy": (None, [_P]),
    "tg_batch_workspace_bytes": (_I, [_P, C.POINTER(_SZ)]),
    "tg_batch_bind_workspace": (_I, [_P, _P, _SZ]),
    "tg_batch_set_density": (_I, [_P, C.POINTER(_P), _D, C.POINTER(_D), _P]),
    "tg_batch_solve": (_I, [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(SolverOpts),
                            C.POINTER(SolveResult), _P]),
    "tg_batch_history": (_I, [_P, _I, _I, C.POINTER(_D), _P]),
    "tg_batch_tile_heights": (_I, [_P, _I, C.POINTER(_I)]),
    "tg_batch_select_floor": (_I, [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(Policy),
                                   C.POINTER(_P), C.POINTER(PolicyResult), _P]),
    "tg_mlp_workspace_bytes": (_I, [_I, C.POINTER(_SZ)]),
    "tg_mlp_create": (_I, [_P, _SZ, _I, C.POINTER(_P)]),
    "tg_mlp_destroy": (None, [_P]),
    "tg_mlp_set_params": (_I, [_P, C.POINTER(C.c_float), C.POINTER(C.c_float),
                               C.POINTER(C.c_float), _P]),
    "tg_mlp_get_params": (_I, [_P, C.POINTER(C.c_float), _P]),
    "tg_mlp_forward": (_I, [_P, _P, _I, _P, _P]),
    "tg_mlp_train_step": (_I, [_P, _P, _P, _I, C.c_float, C.POINTER(C.c_float), _P, _P]),
    "tg_density_features": (_I, [_P, _P, _D, _D, C.POINTER(_D), _P]),
    "tg_batch_autotune": (_I, [_P, _I, _I, C.POINTER(_I), C.POINTER(_D), _P]),
    "tg_autotune": (_I, [_P, _I, _I, C.POINTER(_I), C.POINTER(_D), _P]),
    "tg_compliance_sensitivity": (_I, [_P, _P, _D, _D, _P, _P, _P, _P, C.POINTER(_D), _P]),
    "tg_gradient_change": (_I, [_P, _P, _D, _P, _P, C.POINTER(GradientChange), _P]),
    "tg_gradient_change_noalloc": (_I, [C.c_int64, _P, _D, _P, _P, C.POINTER(GradientChange), _P]),
    "tg_density_filter": (_I, [_P, _P, _D, _P, _P]),
    "tg_density_filter_adjoint": (_I, [_P, _P, _P, _D, _P, _P]),
    "tg_filter_project": (_I, [_P, _P, _D, _D, _D, _P, _P, _P, _P]),
    "tg_oc_update": (_I, [_P, _P, _P, _P, _D, _D, _D, _D, _D, _P, C.POINTER(_D), _P]),
    "tg_default_topopt": (None, [C.POINTER(TopoptOpts)]),
    "tg_topopt_workspace_bytes": (_I, [_P, C.POINTER(_SZ)]),
    "tg_topopt_run": (_I, [_P, _P, C.POINTER(TopoptOpts), _P, _SZ, _P, C.POINTER(TopoptRecord),
                           C.POINTER(_I), _P]),
    "tg_spectrum_workspace_bytes": (_I, [_P, C.POINTER(_SZ)]),
    "tg_adaptive_workspace_bytes": (_I, [_P, _I, _I, C.POINTER(_SZ)]),
    "tg_adaptive_precondition": (_I, [_P, _P, _P, _I, _I, _P, _SZ, C.POINTER(_I), _P]),
    "tg_adaptive_solve": (_I, [_P, _P, _P, C.POINTER(SolverOpts), _I, _P, _SZ, C.POINTER(SolveResult),
                               C.POINTER(_D), C.POINTER(_I), C.POINTER(_I), _P]),
    "tg_adaptive_checkpoints": (_I, [_P, _P, _P, C.POINTER(SolverOpts), _I, _I, _I, _P, _SZ,
                                     C.POINTER(SolveResult), C.POINTER(_I), C.POINTER(_D), C.POINTER(_D),
                                     C.POINTER(_I), _P]),
    "tg_default_stack_opts": (None, [C.POINTER(StackOpts)]),
    "tg_stack_workspace_bytes": (_I, [_P, _I, C.POINTER(StackOpts), C.POINTER(_SZ)]),
    "tg_stack_lambdas": (_I, [_P, C.POINTER(StackOpts), _P, _SZ, C.POINTER(_D), _P]),
    "tg_stack_precondition": (_I, [_P, _P, _P, C.POINTER(StackOpts), C.POINTER(_D), _P, _SZ, C.POINTER(StackLog),
                                   _P]),
    "tg_stack_solve": (_I, [_P, _P, _P, C.POINTER(SolverOpts), C.POINTER(StackOpts), _P, _SZ,
                            C.POINTER(SolveResult), C.POINTER(_D), C.POINTER(StackLog), C.POINTER(_I),
                            C.POINTER(_D), _P]),
    "tg_stack_select_floor": (_I, [_P, _P, _P, C.POINTER(Policy), C.POINTER(StackOpts), _P, _SZ, _P,
                                   C.POINTER(PolicyResult), _P]),
    "tg_extreme_eigenvalues": (_I, [_P, _I, _I, _D, _P, _SZ, C.POINTER(SpectrumResult), _P]),
    "tg_timer_enable": (_I, [_I]),
    "tg_timer_reset": (_I, []),
    "tg_timer_read": (_I, [_I, C.POINTER(_D), C.POINTER(C.c_longlong), C.POINTER(_D)]),
    "tg_timer_name": (C.c_char_p, [_I]),
}
TG_KT_COUNT = 9
TG_AD_MAX_RESTART = 512
TG_NOALLOC_SCRATCH_BYTES, TG_NOALLOC_MAX_ELEMS = 49264, 2147483647


def header_symbols(path=HEADER):
    """Function names declared in the public header."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tg_[A-Za-z0-9_]+)\s*\(", text)))


_lib = None


class TopoguardError(RuntimeError):
    pass


def lib():
    """Load the built library (raises if it is missing: no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TopoguardError(
            f"{LIB_PATH} not found: build it with __graft_entry__.build() "
            "(python -m paper_2607_26382_amd.build)")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(rc):
    if rc != 0:
        msg = lib().tg_last_error().decode(errors="replace")
        raise TopoguardError(f"topoguard error {rc}: {msg}")
    return rc
