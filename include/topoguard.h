/*
 * topoguard - guarded matrix-free SIMP state solve for AMD MI355X (gfx950).
 *
 * C ABI of libtopoguard.so.  Every call follows the statement of the problem
 * in arXiv 2607.26382 ("When a positive SIMP density floor is not enough"):
 *
 *   K(rho_min) u = f,  K(rho_min) = sum_e E_e K_e  on the free DOFs
 *   (Eq. frozen_operator), E_e = rho_min + (1 - rho_min) rho_e^p
 *   (Eq. floor_scaling), acceptance only on the recomputed FP64 relative
 *   residual eta = ||f - K u|| / ||f|| <= tau (Eq. relative_residual,
 *   Tab. residual-semantics), floor chosen by the probe -> two-feature rule ->
 *   guarded ladder of Alg. floor_policy.
 *
 * Conventions for every function:
 *   - return 0 on success; a negative TG_E* code on failure, with a message
 *     available from tg_last_error() (thread-local, valid until the next call
 *     on the same thread).  Solver non-convergence is an OUTCOME reported in
 *     a result struct, never an error code.
 *   - "_d" pointers are device pointers (HIP global memory on the current
 *     device); "_h" pointers are host pointers.  The library never keeps a
 *     caller pointer beyond the call, except the workspace bound with
 *     tg_bind_workspace / tg_batch_bind_workspace, which the caller owns and
 *     must keep alive (and unmoved) until the handle is destroyed.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *     device work is enqueued on it.  Functions returning host scalars
 *     synchronize that stream before returning.
 *   - Grid layout: elements e = ex + nx (ey + ny ez) (x fastest); nodes
 *     n = i + (nx+1) (j + (ny+1) k); DOF 3 n + c (c = x, y, z).  Vectors are
 *     full length (3 * n_nodes) and hold 0 on the clamped DOFs (x = 0 face):
 *     inputs there are ignored (treated as 0), outputs there are written 0.
 *   - A handle is not thread-safe; distinct handles may be used concurrently
 *     on distinct streams.
 */
#ifndef TOPOGUARD_H
#define TOPOGUARD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TG_OK = 0,
  TG_EINVAL = -1,      /* invalid argument (sizes, ranges, NaN density, ...) */
  TG_EHIP = -2,        /* a HIP runtime call failed                          */
  TG_EWORKSPACE = -3,  /* workspace missing or too small                     */
  TG_ESTATE = -4,      /* call out of order (e.g. apply before set_density)  */
  TG_ENUMERIC = -5     /* coarsest factorization met a non-positive pivot    */
};

/* Precision of the operator / preconditioner path (addition (1)). */
enum {
  TG_F64 = 0,          /* FP64 vectors and arithmetic                          */
  TG_F32 = 1,          /* FP32 vectors and arithmetic                          */
  TG_BF16MFMA = 2,     /* FP32 vectors; fine-level Ke contraction on BF16
                          matrix cores (inputs rounded to BF16), FP32 accumulate */
  TG_BF16X3MFMA = 3    /* as TG_BF16MFMA with split BF16 (hi + lo) operands:
                          Ke_hi u_hi + Ke_hi u_lo + Ke_lo u_hi, ~16 bits      */
};

/* FGMRES outcomes (the solver's internal flag semantics, Tab. residual-semantics). */
enum {
  TG_PROJ_CONVERGED = 0, /* stopping estimate <= tol (diagnostic only) */
  TG_MAXIT = 1,          /* iteration cap reached                      */
  TG_BREAKDOWN = 2,      /* Hessenberg subdiagonal collapsed           */
  TG_NONFINITE = 3       /* a non-finite scalar appeared               */
};

/* Multigrid options (Tab. solver-config, fixed linear V-cycle). */
typedef struct {
  int max_levels;      /* 0 = automatic: coarsen 2:1 while dims even, >= 2, and free DOF > max_coarse_dof */
  int max_coarse_dof;  /* default 300                                   */
  double omega;        /* node-block Jacobi damping, default 0.6        */
  int nu_pre, nu_post; /* sweeps, default 2 / 2                         */
} tg_mg_opts;

/* FGMRES options. */
typedef struct {
  int restart;         /* m, default 30                                 */
  int max_iters;       /* cap across restarts, default 200              */
  double tol;          /* stopping tolerance on the history value, 1e-6 */
  int prec;            /* preconditioner precision TG_F64/F32/BF16MFMA  */
  int cgs_passes;      /* 1 = CGS; 2 = CGS2 with the reorthogonalization
                          delayed into the next step (default: two sweeps
                          over the basis per step); 3 = CGS2 in place
                          (three sweeps per step)                        */
  double breakdown;    /* subdiagonal <= breakdown * ||w|| -> BREAKDOWN, 1e-14 */
  int graphs;          /* nonzero: each run of Arnoldi steps between two
                          status reads (V-cycle, K z, Gram-Schmidt sweeps,
                          scalar kernels) is captured once as a HIP graph
                          per work-list state and step range and replayed;
                          results are bitwise those of direct launches.
                          Default 0.                                     */
  int sync_every;      /* Arnoldi steps between host reads of the per-
                          problem status, >= 1 (default 8).  The kernels of
                          a step skip problems whose status on the device is
                          no longer running, so a problem that stops inside
                          a run of steps is left exactly as if the run had
                          ended there: results are bitwise the same for
                          every value.  Checkpointed solves read after every
                          step.                                          */
} tg_solver_opts;

typedef struct {
  int iterations;      /* total FGMRES iterations                        */
  int outcome;         /* TG_PROJ_CONVERGED / TG_MAXIT / ...             */
  double proj_eta;     /* last history value (stopping estimate)         */
  double true_eta;     /* recomputed FP64 relative residual (guard) or -1 */
} tg_solve_result;

typedef struct {
  int nx, ny, nz;          /* fine elements                                  */
  int64_t n_elem, n_nodes, n_dof, n_free;
  int n_levels;
  int level_dims[8][3];    /* elements per level                             */
  int coarse_free_dof;     /* free DOFs of the coarsest level                */
} tg_grid_info;

typedef struct tg_grid tg_grid;
typedef struct tg_batch tg_batch;
typedef struct tg_mlp tg_mlp;

/* ---- errors, defaults -------------------------------------------------- */
const char* tg_last_error(void);
void tg_default_mg_opts(tg_mg_opts* o);
void tg_default_solver_opts(tg_solver_opts* o);

/* ---- grid (Sec. 3.1: structured cubic hex8 grid, one shared Ke) ---------- */
/* Builds the host Ke (E0, nu, unit cube, 2x2x2 Gauss), index maps, hierarchy
 * dimensions.  Cantilever boundary: x = 0 face clamped.  mg may be NULL
 * (defaults).  No device memory is touched until a workspace is bound. */
int tg_setup_grid(int nx, int ny, int nz, double E0, double nu,
                  const tg_mg_opts* mg, tg_grid** out);
void tg_destroy(tg_grid* g);
int tg_get_grid_info(const tg_grid* g, tg_grid_info* info);
/* Copies the 24x24 FP64 element stiffness (row-major, local node
 * a = i + 2j + 4k, DOF 3a + c) to ke_h. */
int tg_get_ke(const tg_grid* g, double* ke_h);
/* Unit -z load on the x = L, z = 0 edge by tributary length (total -1),
 * written to the full-length host vector f_h (3 * n_nodes doubles). */
int tg_edge_load(const tg_grid* g, double* f_h);

/* Device workspace for one grid: every device array the grid and its solver
 * use (moduli, coarse operators, smoother blocks, coarsest inverse, Krylov
 * bases for restart <= max_restart, V-cycle vectors).  The caller allocates
 * `bytes` (256-byte aligned) and binds it. */
int tg_workspace_bytes(const tg_grid* g, int max_restart, size_t* bytes);
int tg_bind_workspace(tg_grid* g, void* ws_d, size_t bytes, int max_restart);

/* ---- density (Eq. floor_scaling) ---------------------------------------- */
/* rho_d: n_elem FP64 stored densities in [0,1] (device).  p > 0,
 * 0 < rho_min <= 1.  Builds E_e (FP64 and FP32), Galerkin coarse operators,
 * node-block smoother inverses and the coarsest dense inverse.  Synchronizes
 * `stream` (validation).  TG_EINVAL on a non-finite or out-of-range density. */
int tg_set_density(tg_grid* g, const double* rho_d, double p, double rho_min, void* stream);

/* ---- operator (Eq. frozen_operator) -------------------------------------- */
/* y = K(rho_min) u on the free DOFs.  prec TG_F64: u_d, y_d are double;
 * TG_F32 / TG_BF16MFMA / TG_BF16X3MFMA: float.  Needs tg_set_density first
 * (TG_ESTATE). */
int tg_apply_K(const tg_grid* g, const void* u_d, void* y_d, int prec, void* stream);

/* ---- preconditioner (Tab. solver-config, fixed V-cycle) ------------------ */
/* z = M^-1 r: one fixed linear V-cycle.  Vector dtype follows prec as above. */
int tg_vcycle(tg_grid* g, const void* r_d, void* z_d, int prec, void* stream);

/* ---- solve (right-preconditioned FGMRES, Sec. 3.5) ------------------------ */
/* x0 = 0.  f_d, u_d: double.  hist_h (may be NULL) receives iterations+1
 * history values (cycle-start true residuals, in-cycle projected estimates).
 * res->true_eta is -1 (the guard is a separate call). */
int tg_fgmres_solve(tg_grid* g, const double* f_d, double* u_d, const tg_solver_opts* o,
                    tg_solve_result* res, double* hist_h, void* stream);

/* ---- guard (Eq. relative_residual; Alg. floor_policy acceptance) ---------- */
/* eta = ||f - K u||_2 / ||f||_2 over free DOFs in FP64. */
int tg_true_residual(const tg_grid* g, const double* f_d, const double* u_d,
                     double* eta_h, void* stream);

/* ---- probe (Sec. 3.4) ------------------------------------------------------ */
/* Runs FGMRES at the current floor for at most `iters` iterations with restart
 * o->restart (the caller passes restart >= iters for one-cycle semantics) and
 * returns r50 = hist[min(50,k_stop)], r100 = hist[min(100,k_stop)]. */
int tg_probe_features(tg_grid* g, const double* f_d, const tg_solver_opts* o, int iters,
                      double* r50_h, double* r100_h, int* k_stop_h, void* stream);

/* The probe with periodic true-residual checkpoints (the detector variant
 * Sec. 4.1.1 leaves untested): the same FGMRES as tg_probe_features, and
 * after every `every` iterations the FP64 relative residual of the current
 * iterate x_k = x_0 + Z_k y_k (y_k the least-squares solution over the
 * columns so far) is recomputed without changing the iteration.  For the
 * first min(cap, count) checkpoints: k_h[i] = k, true_h[i] = that residual,
 * proj_h[i] = the history value at k (the projected estimate, or the
 * cycle-start true residual at a restart boundary).  *n_h = number written.
 * Not with o->graphs.  Synchronizes `stream`. */
int tg_probe_checkpoints(tg_grid* g, const double* f_d, const tg_solver_opts* o, int iters, int every, int cap,
                         int* k_h, double* proj_h, double* true_h, int* n_h, int* k_stop_h, void* stream);

/* ---- adaptive preconditioner (Tab. solver-config, fine-level correction) -- */
/* One application z = M(v): one V-cycle at precision `prec` (z = V(v)), then
 * the fine-level correction: with s = v - K z, `inner_steps` steps of
 * right-preconditioned GMRES (restart = inner_steps, CGS2, no tolerance stop)
 * on K d = s from d = 0, preconditioned by the 3 x 3 node-block Jacobi
 * operator (the inverses of K's diagonal node blocks); z + d replaces z only
 * if ||s - K d||_2 < ||s||_2.  inner_steps = 0 is the plain V-cycle.  K is
 * the FP64 operator in every precision.  The outer method must be flexible
 * (Sec. 3.5): M is nonlinear in v.
 * Single grid; the outer iteration reads each Arnoldi column back to the host,
 * one application of M needs no host synchronization;
 * FP64 vectors of n_dof entries (device), clamped DOFs read as 0 and written
 * as 0.  The caller allocates the workspace (tg_adaptive_workspace_bytes with
 * the outer restart, 0 for tg_adaptive_precondition) and keeps ownership.
 * Errors: TG_ESTATE before tg_set_density, TG_EINVAL for a NULL vector, a
 * precision outside TG_F64..TG_BF16X3MFMA or restart / inner_steps outside
 * [0, TG_AD_MAX_RESTART], TG_EWORKSPACE for a short workspace.  Both calls
 * synchronize `stream`. */
#define TG_AD_MAX_RESTART 512
int tg_adaptive_workspace_bytes(const tg_grid* g, int restart, int inner_steps, size_t* bytes);
/* v_d and z_d must not overlap; *accepted_h (may be NULL) = 1 if the correction
 * was kept. */
int tg_adaptive_precondition(tg_grid* g, const double* v_d, double* z_d, int prec, int inner_steps, void* ws_d,
                             size_t ws_bytes, int* accepted_h, void* stream);
/* FGMRES (o->restart >= 1, o->max_iters, o->tol, o->breakdown; cgs_passes 1
 * = CGS, otherwise CGS2 in place; o->graphs ignored) preconditioned by M,
 * with the history semantics of tg_fgmres_solve: hist_h (may be NULL, room
 * for max_iters + 1) receives iterations + 1 values.  accepted_h (may be NULL,
 * room for max_iters + 1) receives, per application of M in order, 1 if its
 * correction was kept; *n_applied_h (may be NULL) = the number of
 * applications.  x0 = 0; f_d and u_d must not overlap; res->true_eta = -1 (the
 * guard is tg_true_residual). */
int tg_adaptive_solve(tg_grid* g, const double* f_d, double* u_d, const tg_solver_opts* o, int inner_steps,
                      void* ws_d, size_t ws_bytes, tg_solve_result* res, double* hist_h, int* accepted_h,
                      int* n_applied_h, void* stream);
/* tg_adaptive_solve with periodic true-residual checkpoints (the detector
 * variant Sec. 4.1.1 leaves untested, here under the adaptive preconditioner):
 * after every `every` (>= 1) iterations the FP64 relative residual of the
 * current iterate x_k = x_0 + Z_k y_k is recomputed without changing the
 * iteration.  For the first min(cap, count) checkpoints: k_h[i] = k,
 * proj_h[i] = the history value at k, true_h[i] = that residual; *n_h = number
 * written.  u_d receives the solution as in tg_adaptive_solve. */
int tg_adaptive_checkpoints(tg_grid* g, const double* f_d, double* u_d, const tg_solver_opts* o, int inner_steps,
                            int every, int cap, void* ws_d, size_t ws_bytes, tg_solve_result* res, int* k_h,
                            double* proj_h, double* true_h, int* n_h, void* stream);

/* ---- the full adaptive stack (Tab. solver-config; Sec. 3.5) --------------- */
/* One application z = M(v), every part in FP64 on the device:
 *   1. Chebyshev smoothing of degree nu_pre on K x = v from x = 0, on the
 *      interval [lo, hi] * lambda~ of the finest level;
 *   2. r = v - K x; the coarse problem K_1 e = P^T r (K_1 the Galerkin
 *      operator of level 1, P the trilinear prolongation) gets coarse_steps
 *      steps of GMRES (restart = coarse_steps, CGS2, no tolerance stop) from
 *      e = 0, right-preconditioned by the V-cycle of levels 1.. with
 *      Chebyshev smoothing (coarse_steps = 0: one such V-cycle; level 1
 *      coarsest: the direct solve);
 *   3. line search: with d = P e, alpha = (r . K d) / (K d . K d) (0 if
 *      K d = 0) minimizes ||r - alpha K d||_2; the correction x += alpha d
 *      is kept iff ratio = ||r - alpha K d|| / ||r|| <= theta (ratio = 1
 *      when r = 0);
 *   4. Chebyshev smoothing of degree nu_post from x;
 *   5. the fine-level correction of tg_adaptive_precondition (inner_steps
 *      GMRES steps with the node-block Jacobi preconditioner, kept iff it
 *      lowers ||v - K z||).
 * The Chebyshev iteration x_{k+1} = x_k + omega_k D^-1 (b - K x_k) +
 * beta_k (x_k - x_{k-1}) (D the 3 x 3 node blocks of the level's operator)
 * targets [lo, hi] * lambda~_l, where lambda~_l = ||D^-1 K v|| after
 * power_iters normalized power steps from the start vector v_d =
 * ((d + 1) * 0x9E3779B1 mod 2^32) / 2^32 - 0.5 over the level's free DOFs d
 * (full numbering: x-fastest nodes, three components).  The outer method
 * must be flexible: M is nonlinear in v.
 * Single grid with at least two levels; vectors: FP64, n_dof entries
 * (device), clamped DOFs read as 0 and written as 0.  The caller allocates
 * the workspace (tg_stack_workspace_bytes with the outer restart, 0 for
 * tg_stack_precondition / tg_stack_lambdas) and keeps ownership; the grid's
 * own level vectors are used as scratch.
 * Errors: TG_ESTATE before tg_set_density, TG_EINVAL for NULL arguments, a
 * single-level grid, steps outside [0, TG_AD_MAX_RESTART], degrees outside
 * [1, 16], power_iters outside [1, 1000], not 0 < lo < hi, or theta < 0;
 * TG_EWORKSPACE for a short workspace.  Every call synchronizes `stream`. */
typedef struct {
  int inner_steps;     /* fine-level correction steps, default 20 (0: none)  */
  int coarse_steps;    /* level-1 GMRES steps, default 10                     */
  int nu_pre, nu_post; /* Chebyshev degrees, default 2 / 2                    */
  int power_iters;     /* power steps for lambda~, default 10                 */
  double lo, hi;       /* Chebyshev interval factors, default 0.1 / 1.1       */
  double theta;        /* acceptance ratio of the coarse correction, 0.95     */
} tg_stack_opts;
typedef struct {
  double alpha;        /* line-search step of the coarse correction           */
  double ratio;        /* ||r - alpha K d|| / ||r||                           */
  int coarse_accepted; /* ratio <= theta                                      */
  int fine_kept;       /* the fine-level correction was kept                  */
} tg_stack_log;
void tg_default_stack_opts(tg_stack_opts* so);
int tg_stack_workspace_bytes(const tg_grid* g, int restart, const tg_stack_opts* so, size_t* bytes);
/* lams_h (room for n_levels - 1): lambda~ of every level above the coarsest. */
int tg_stack_lambdas(tg_grid* g, const tg_stack_opts* so, void* ws_d, size_t ws_bytes, double* lams_h,
                     void* stream);
/* z = M(v); v_d and z_d must not overlap.  lams_h: lambda~ per level (n_levels
 * - 1 values > 0) or NULL to estimate them first.  *log_h (may be NULL)
 * receives the application's decisions. */
int tg_stack_precondition(tg_grid* g, const double* v_d, double* z_d, const tg_stack_opts* so,
                          const double* lams_h, void* ws_d, size_t ws_bytes, tg_stack_log* log_h, void* stream);
/* FGMRES preconditioned by M (options and history as in tg_adaptive_solve;
 * o->prec is not used: the stack runs in FP64).  lambda~ is estimated once
 * per call.  log_h (may be NULL, room for max_iters + 1) receives one entry
 * per application of M in order, *n_applied_h (may be NULL) their number,
 * lams_h (may be NULL, room for n_levels - 1) the estimates used. */
int tg_stack_solve(tg_grid* g, const double* f_d, double* u_d, const tg_solver_opts* o, const tg_stack_opts* so,
                   void* ws_d, size_t ws_bytes, tg_solve_result* res, double* hist_h, tg_stack_log* log_h,
                   int* n_applied_h, double* lams_h, void* stream);

/* ---- policy (Alg. floor_policy) ------------------------------------------ */
enum { TG_SELECT_RULE = 0, TG_SELECT_MLP = 1, TG_SELECT_FIXED = 2 };
#define TG_MAX_RUNGS 8
typedef struct {
  int n_rungs;                   /* rungs[0] = original floor rho_0            */
  double rungs[TG_MAX_RUNGS];    /* increasing floors, e.g. 1e-9,1e-6,1e-4,1e-3 */
  double p;                      /* SIMP exponent                              */
  double tau;                    /* guard tolerance, 1e-6                      */
  int probe_iters;               /* 100                                        */
  int probe_restart;             /* 100                                        */
  double t_high, t_plateau, t_ratio;   /* Eq. trigger: 1e-2, 1e-4, 0.6      */
  int selector;                  /* TG_SELECT_*                                */
  int fixed_rung;                /* for TG_SELECT_FIXED                        */
  const tg_mlp* mlp;             /* for TG_SELECT_MLP (rule if NULL)           */
  tg_solver_opts solve;          /* per-rung solves (restart 30, cap 200, ...) */
  int want_features;             /* nonzero: fill the six density statistics of
                                    tg_policy_result.features with any selector */
} tg_policy;

typedef struct {
  int rung;                      /* accepted rung index, -1 = none admissible */
  double floor;                  /* accepted floor or -1                      */
  int k0;                        /* first attempted rung                      */
  double r50, r100;              /* probe features                            */
  int probe_iters;               /* k_stop of the probe                       */
  int n_attempts;
  struct {
    int rung, iterations, outcome, accepted;
    double floor, proj_eta, true_eta;
  } attempts[TG_MAX_RUNGS];
  int iters_probe, iters_selected, iters_rejected;   /* stage accounting      */
  double features[8];            /* selector input (log r50, log r100, 6 stats) */
} tg_policy_result;

void tg_default_policy(tg_policy* pol);
/* rho_d: stored densities (device).  On return u_d holds the accepted
 * solution (zeros if rung == -1).  Never returns a solution whose FP64
 * eta > tau. */
int tg_select_floor(tg_grid* g, const double* rho_d, const double* f_d, const tg_policy* pol,
                    double* u_d, tg_policy_result* out, void* stream);
/* Alg. floor_policy with the adaptive stack preconditioning every solve
 * (the paper's own configuration, Tab. solver-config): the probe at
 * pol->rungs[0] (pol->probe_iters iterations, restart pol->probe_restart,
 * tolerance pol->solve.tol), the first rung from Eq. trigger, the network or a
 * fixed rung as in tg_select_floor, then per rung from there an independent
 * tg_stack_solve with pol->solve's restart, cap and tolerance, followed by the
 * FP64 guard eta = ||f - K u|| / ||f|| <= pol->tau (Eq. relative_residual);
 * the first accepted rung ends the climb.  pol->solve.prec is not used (the
 * stack runs in FP64).  Single grid with at least two levels; rho_d: stored
 * densities (device, n_elem doubles), f_d and u_d: FP64, n_dof (device).  On
 * return u_d holds the accepted solution, or zeros when no rung is accepted;
 * the probe's iterate is never returned.  Workspace: tg_stack_workspace_bytes
 * with max(probe_restart, solve.restart), caller-owned.  Errors as
 * tg_stack_solve and tg_select_floor; synchronizes `stream`. */
int tg_stack_select_floor(tg_grid* g, const double* rho_d, const double* f_d, const tg_policy* pol,
                          const tg_stack_opts* so, void* ws_d, size_t ws_bytes, double* u_d,
                          tg_policy_result* out, void* stream);

/* ---- batching (addition (2)) --------------------------------------------- */
/* A batch solves independent problems of possibly different grid sizes
 * together: every kernel launch covers all active problems.  Each grid keeps
 * its own bound workspace; the batch needs a small workspace of its own. */
int tg_batch_create(int n, tg_grid* const* grids, tg_batch** out);
void tg_batch_destroy(tg_batch* b);
int tg_batch_workspace_bytes(const tg_batch* b, size_t* bytes);
int tg_batch_bind_workspace(tg_batch* b, void* ws_d, size_t bytes);
/* rho_d[i], rho_min[i] per problem; p shared. */
int tg_batch_set_density(tg_batch* b, const double* const* rho_d, double p,
                         const double* rho_min_h, void* stream);
/* f_d[i] -> u_d[i]; res[i] gets the outcome and (guard) true_eta. */
int tg_batch_solve(tg_batch* b, const double* const* f_d, double* const* u_d,
                   const tg_solver_opts* o, tg_solve_result* res, void* stream);
/* History of problem i of the last tg_batch_solve on this batch (the same
 * values tg_fgmres_solve returns in hist_h: cycle-start true residuals and
 * in-cycle projected estimates, Tab. residual-semantics): `count` doubles,
 * count <= res[i].iterations + 1 is meaningful, count <= 4096 accepted.
 * Synchronizes `stream`.  TG_EINVAL for i or count out of range. */
int tg_batch_history(const tg_batch* b, int i, int count, double* hist_h, void* stream);
/* Alg. floor_policy for every problem at once (probe, first rung, ladder). */
int tg_batch_select_floor(tg_batch* b, const double* const* rho_d, const double* const* f_d,
                          const tg_policy* pol, double* const* u_d, tg_policy_result* out,
                          void* stream);

/* ---- autotuner (addition (2)) -------------------------------------------- */
/* Times the V-cycle smoothing sweep of the matrix-free levels for each
 * candidate z-tile height and keeps the fastest per level: the tile height
 * trades one redundant element layer per tile against parallelism and
 * against the last, partly filled round of resident workgroups.  Candidates:
 * 2, 3, 4, 6, 8 and every balanced height ceil(NZ / t), t = 1..64, of the
 * batch's grids at that level.  Needs set_density.  zc_out (may be NULL) receives the 8
 * per-level heights, us_out (may be NULL) the best sweep time per level in
 * microseconds (-1 where nothing was timed).  Choices are cached per batch
 * signature (grid sizes in order, precision) for the process and, if the
 * environment variable TG_AUTOTUNE_CACHE names a file, across runs; a cached
 * choice is applied without timing unless force is nonzero.  Tile heights
 * change only the work decomposition: results agree with untuned runs to
 * rounding.  Synchronises the stream; TG_ESTATE before set_density. */
int tg_batch_autotune(tg_batch* b, int prec, int force, int* zc_out, double* us_out, void* stream);
/* The z-tile heights (node layers per tile) problem i of the batch uses at
 * each of its levels (zc_out: 8 ints, 0 beyond its levels).  In a batch of
 * several grid sizes the autotuner picks them per size: after the level-wide
 * choice it revisits each size in turn, the others fixed, timing the sweep
 * over the whole batch.  TG_EINVAL for i out of range. */
int tg_batch_tile_heights(const tg_batch* b, int i, int* zc_out);
int tg_autotune(tg_grid* g, int prec, int force, int* zc_out, double* us_out, void* stream);

/* ---- learned first-floor selector (addition (4)) ------------------------- */
/* 8 -> 64 -> 64 -> 4 MLP, exact-erf GELU, softmax cross-entropy, Adam
 * (beta = 0.9, 0.999, eps = 1e-8).  Input: log10 r50, log10 r100 and the six
 * density statistics below, standardized as (x - mean) / std; output: logits
 * over the ladder rungs, argmax with ties to the lower rung.  Parameters,
 * optimizer state and staging live in the caller-bound workspace; max_batch
 * bounds the selector's internal batch (forward/train take any B, train
 * reduces over at most 256 per-wave partials).  set_params resets Adam. */
int tg_mlp_workspace_bytes(int max_batch, size_t* bytes);
int tg_mlp_create(void* ws_d, size_t bytes, int max_batch, tg_mlp** out);
void tg_mlp_destroy(tg_mlp* m);
/* params_h: 4996 floats in order W1[64][8], b1[64], W2[64][64], b2[64],
 * W3[4][64], b3[4]; mean_h/std_h: 8 feature standardization constants. */
int tg_mlp_set_params(tg_mlp* m, const float* params_h, const float* mean_h, const float* std_h,
                      void* stream);
int tg_mlp_get_params(const tg_mlp* m, float* params_h, void* stream);
/* x_d: B x 8 raw features (float, device) -> logits_d: B x 4. */
int tg_mlp_forward(const tg_mlp* m, const float* x_d, int B, float* logits_d, void* stream);
/* One Adam step on the mean cross-entropy of (x_d, y_d); loss_h may be NULL.
 * grads_d (may be NULL) receives the 4996 parameter gradients. */
int tg_mlp_train_step(tg_mlp* m, const float* x_d, const int* y_d, int B, float lr,
                      float* loss_h, float* grads_d, void* stream);
/* The six density statistics of a stored density field rho_d (device, n_e
 * doubles, x-fastest) at probe floor rho0 into stats_h[6]: fraction of voxels
 * at 0, mean, smallest nonzero value (0 if none), log10(E_max/E_min) over the
 * nonzero voxels, fraction of the loaded-edge elements (ex = nx-1, ez = 0)
 * 6-connected through {rho >= 0.5} to an element with ex = 0, and
 * log10(n_DOF).  Uses the grid's own label scratch; synchronises the stream. */
int tg_density_features(tg_grid* g, const double* rho_d, double p, double rho0, double* stats_h,
                        void* stream);

/* ---- operator fidelity (Sec. 3.1 sensitivities; Sec. 4.4.1, Tab. perturbation) */
/* For a displacement u_d (full length, double; clamped DOFs read as 0) on
 * this grid:
 *   energy_d[e] = u_e^T K_e u_e                       (may be NULL)
 *   dc_d[e]     = -p (1 - rho_min) rho_e^(p-1) u_e^T K_e u_e, the compliance
 *                 sensitivity dC/drho_e of Sec. 3.1 at the densities rho_d
 *                 (n_elem doubles, the densities that enter Eq. floor_scaling;
 *                 used as given, not validated)       (may be NULL)
 *   *compliance_h = f^T u over the free DOFs (f_d full length, double)
 *                 (may be NULL; then f_d may be NULL too)
 * p > 0 and 0 <= rho_min <= 1 are those of the solve u came from; they need
 * not match the last set_density.  At least one output must be requested.
 * Works in FP64 in a fixed summation order (bitwise reproducible); uses the
 * grid's reduction scratch, so it must not overlap another call on the same
 * grid.  Synchronizes `stream` when compliance_h is requested. */
int tg_compliance_sensitivity(const tg_grid* g, const double* rho_d, double p, double rho_min,
                              const double* f_d, const double* u_d, double* energy_d, double* dc_d,
                              double* compliance_h, void* stream);

typedef struct {
  int64_t n_solid;     /* elements with rho >= solid_min                      */
  double rel_l2;       /* ||g1 - g0|| / ||g0|| over those elements             */
  double pearson;      /* Pearson correlation of g0 and g1 over them (NaN if
                          either is constant there)                           */
  double norm0, norm1; /* ||g0||, ||g1|| over them                             */
} tg_gradient_change_result;

/* The gradient columns of Tab. perturbation: two sensitivity fields dc0_d
 * (reference floor) and dc1_d (raised floor), n_elem doubles each, compared
 * over the solid elements rho_d[e] >= solid_min (two FP64 passes: sums, then
 * centred sums; fixed order).  TG_EINVAL if no element is solid.
 * Synchronizes `stream`. */
int tg_gradient_change(const tg_grid* g, const double* rho_d, double solid_min, const double* dc0_d,
                       const double* dc1_d, tg_gradient_change_result* out, void* stream);

/* ---- allocation-free entry point ------------------------------------------
 * For callers that cannot allocate device memory or bind a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same comparison as tg_gradient_change (same kernels, same
 * summation order, so bitwise the same result) on n_elem elements, with no
 * grid: rho_d, dc0_d, dc1_d are device arrays of n_elem doubles, `out` a host
 * struct.  The reduction partials live in a fixed array inside the library,
 * TG_NOALLOC_SCRATCH_BYTES per GPU, taken when the library is loaded and held
 * until the process ends; the call allocates nothing (no hipMalloc, no host
 * heap).  Every call on one GPU shares that GPU's array and rewrites every
 * value it reads, so calls in sequence are independent, but calls that
 * overlap on one GPU (two host threads, or two streams without ordering)
 * race and give undefined results.  Any n_elem in [1, TG_NOALLOC_MAX_ELEMS]
 * fits the array (the partial sums come from at most 1024 workgroups);
 * larger or smaller counts, NULL pointers and a non-finite solid_min are
 * TG_EINVAL, as is no element with rho >= solid_min.  Synchronizes
 * `stream`. */
#define TG_NOALLOC_SCRATCH_BYTES 49264
#define TG_NOALLOC_MAX_ELEMS 2147483647LL
int tg_gradient_change_noalloc(int64_t n_elem, const double* rho_d, double solid_min, const double* dc0_d,
                               const double* dc1_d, tg_gradient_change_result* out, void* stream);

/* ---- conditioning (Sec. 4.2, Eq. screen) ------------------------------------ */
typedef struct {
  double lambda_min, lambda_max;  /* extreme eigenvalues of K(rho_min), free DOFs   */
  double kappa;                   /* lambda_max / lambda_min                        */
  double resid_min;               /* ||K x - lambda_min x|| / ||K x|| at the end     */
  int iters_min, iters_max;       /* LOBPCG and Lanczos steps taken                 */
  int converged;                  /* resid_min <= tol reached                        */
} tg_spectrum_result;

/* Device workspace of tg_extreme_eigenvalues (7 FP64 and 2 FP32 DOF vectors). */
int tg_spectrum_workspace_bytes(const tg_grid* g, size_t* bytes);
/* Extreme eigenvalues of the operator of the last set_density: lambda_max by
 * Lanczos on K (at most max_iters steps, stopped when the largest Ritz value
 * is stable to 1e-12), lambda_min by LOBPCG preconditioned by one V-cycle at
 * precision prec per step, stopped when ||K x - lambda x|| <= tol ||K x|| or
 * after max_iters steps (converged = 0; lambda_min is then an upper bound).
 * Both start from a fixed hashed vector (deterministic).  The condition
 * number gives the indicator kappa * eps and the screen c eps / tau with
 * c = kappa * rho_min.  Synchronizes `stream` every step; uses the grid's
 * reduction scratch.  TG_ESTATE before set_density. */
int tg_extreme_eigenvalues(tg_grid* g, int prec, int max_iters, double tol, void* ws_d, size_t ws_bytes,
                           tg_spectrum_result* out, void* stream);

/* ---- the optimizer around the solve (Sec. 3.1 Eq. to_problem, Eq. projection;
 *      Sec. 4.1.2; Tab. trajectory-settings) ------------------------------- */
/* Element fields are n_elem doubles on the device (x fastest).  r_min is the
 * linear-hat filter radius in element widths, 0 < r_min < 4: weights
 * w_ej = max(0, r_min - |c_e - c_j|) over the elements j of the grid,
 * normalized per element.  None of these calls synchronizes except
 * tg_oc_update and tg_topopt_run. */
/* xt_d = H x_d (the density filter). */
int tg_density_filter(const tg_grid* g, const double* x_d, double r_min, double* xt_d, void* stream);
/* y_d = H^T (a_d .* b_d) (b_d may be NULL: ones): the chain rule through the
 * filter.  y_d must not alias a_d or b_d. */
int tg_density_filter_adjoint(const tg_grid* g, const double* a_d, const double* b_d, double r_min, double* y_d,
                              void* stream);
/* xbar_d = project(H x_d) with the smoothed Heaviside of Eq. projection
 * (beta > 0, 0 < eta < 1); xt_d (may be NULL) receives H x_d, dxbar_d (may be
 * NULL) d xbar / d xt. */
int tg_filter_project(const tg_grid* g, const double* x_d, double r_min, double beta, double eta, double* xt_d,
                      double* xbar_d, double* dxbar_d, void* stream);
/* One optimality-criteria step: x_new = clip(x sqrt(max(0, -dc) / (lam dv)),
 * max(0, x - move), min(1, x + move)), with lam halving the bracket [0, 1e9]
 * while (l2 - l1) / (l1 + l2) > 1e-9 (at most 200 halvings) so that the
 * physical volume sum_e project(H x_new)_e meets volfrac * n_elem.  dc_d and
 * dv_d are the gradients of the compliance and of that volume with respect
 * to x.  lambda_h (may be NULL) receives the last multiplier.  Synchronizes
 * `stream` once per halving; uses the grid's reduction scratch. */
int tg_oc_update(const tg_grid* g, const double* x_d, const double* dc_d, const double* dv_d, double volfrac,
                 double move, double r_min, double beta, double eta, double* x_new_d, double* lambda_h,
                 void* stream);

enum {
  TG_LOOP_GUARDED = 0,  /* Alg. floor_policy at every outer iteration          */
  TG_LOOP_REUSE = 1,    /* the previous iteration's accepted floor is solved
                           first and kept if the guard accepts it; otherwise
                           (and at the first iteration) the full policy runs  */
  TG_LOOP_FIXED = 2     /* one fixed floor, no acceptance test (the paper's
                           unguarded controls)                                */
};

typedef struct {
  int max_iters, min_iters;  /* 40, 20                                         */
  double tol;                /* stop after min_iters once max |x_new - x| < tol (0.01) */
  double volfrac;            /* 0.30                                           */
  double r_min, eta;         /* 1.5, 0.5                                       */
  int n_stages;              /* continuation stages (1..4), stage q applies
                                from outer iteration stages[q].first_iter on;
                                stages[0].first_iter must be 1               */
  struct {
    int first_iter;
    double p, beta, move;
  } stages[4];               /* defaults: (1, 1.5, 1, 0.20), (16, 3.5, 4, 0.15) */
  int mode;                  /* TG_LOOP_*                                      */
  double fixed_floor;        /* TG_LOOP_FIXED                                  */
  tg_policy policy;          /* rungs (default 1e-12, 1e-3, 1e-2), rule, solves;
                                its p is replaced by the stage's p            */
} tg_topopt_opts;

typedef struct {
  int iter;
  double p, beta;
  double compliance;         /* f^T u of the iteration's solve                 */
  double volume;             /* mean physical density it solved with           */
  double change;             /* max |x_new - x| of its OC step                 */
  int rung;                  /* accepted rung (-1: fixed mode or none)         */
  double floor;              /* floor of the solve used                        */
  int probed;                /* the full policy (probe) ran                    */
  int solve_iters;           /* FGMRES iterations of the iteration, all attempts */
  double true_eta;           /* FP64 guard value of the solve used             */
  int accepted;              /* 1 guard passed, 0 nothing admissible (the loop
                                stops), -1 not tested (fixed mode)            */
  double ms;                 /* wall time of the iteration                      */
} tg_topopt_record;

void tg_default_topopt(tg_topopt_opts* o);
/* Device workspace of tg_topopt_run for this grid (7 element fields and one
 * displacement vector, 256-byte aligned). */
int tg_topopt_workspace_bytes(const tg_grid* g, size_t* bytes);
/* Runs the loop from the design x_d (in: initial design, out: final design)
 * with load f_d.  rec must hold max_iters records; *n_rec receives the number
 * written.  The loop ends early after min_iters once the change is below tol,
 * or (guarded modes) at an iteration where no floor is admissible (its record
 * has accepted = 0).  Synchronizes `stream` repeatedly. */
int tg_topopt_run(tg_grid* g, const double* f_d, const tg_topopt_opts* o, void* ws_d, size_t ws_bytes,
                  double* x_d, tg_topopt_record* rec, int* n_rec, void* stream);

/* ---- instrumentation ----------------------------------------------------- */
/* Kernel-class timer (process-wide): for every class whose bit is set in the
 * mask given to tg_timer_enable (bit k = class k; 0 disables), each launch is
 * bracketed by two HIP events on its own stream and its algorithmic HBM bytes
 * (compulsory reads + writes of the launch, no cache reuse assumed) are
 * accumulated.  tg_timer_read harvests (synchronizes on) the recorded events.
 * Instrumentation only: not part of the method. */
enum {
  TG_KT_APPLY_F64 = 0,       /* fine-level FP64 operator: Arnoldi K z, residuals, guard */
  TG_KT_VCYCLE_FINE = 1,     /* fine-level operator kernels inside the V-cycle          */
  TG_KT_VCYCLE_COARSE = 2,   /* coarse-level operator kernels inside the V-cycle        */
  TG_KT_TRANSFER = 3,        /* restriction, prolongation, first sweep, coarsest solve  */
  TG_KT_MULTIDOT = 4,        /* Gram-Schmidt multi-dot partials                         */
  TG_KT_UPDATE = 5,          /* vector updates (w -= V h, x += Z y, scaling)            */
  TG_KT_SCALAR = 6,          /* reductions and per-problem scalar kernels               */
  TG_KT_SETUP = 7,           /* set_density kernels                                     */
  TG_KT_FIDELITY = 8,        /* compliance, sensitivities, gradient comparison          */
  TG_KT_COUNT = 9
};
int tg_timer_enable(int mask);
int tg_timer_reset(void);
int tg_timer_read(int kind, double* total_ms, long long* launches, double* bytes);
const char* tg_timer_name(int kind);

#ifdef __cplusplus
}
#endif
#endif
