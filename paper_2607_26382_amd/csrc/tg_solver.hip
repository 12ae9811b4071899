// Solver drivers: set_density, FGMRES, true-residual guard, probe and the
// guarded floor ladder, for a batch of problems (a single grid is a batch of
// one).  Host code only sequences kernels and reads per-problem status words.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "tg_internal.h"

namespace tg {

static hipStream_t S(void* s) { return (hipStream_t)s; }

static std::vector<int> all_of(const Batch* b) {
  std::vector<int> v(b->n);
  for (int i = 0; i < b->n; ++i) v[i] = i;
  return v;
}

// E, Galerkin hierarchy, smoother blocks, coarsest inverse for the problems in
// `which`, each with its own density pointer and floor.
int set_density_batch(Batch* b, const std::vector<int>& which, const double* const* rho_d,
                      double p, const double* rho_min, hipStream_t s) {
  if (!(p > 0) || !std::isfinite(p)) return fail(TG_EINVAL, "SIMP exponent p must be > 0");
  for (int q = 0; q < (int)which.size(); ++q) {
    const int i = which[q];
    if (!(rho_min[q] > 0.0 && rho_min[q] <= 1.0)) return fail(TG_EINVAL, "rho_min must be in (0, 1]");
    if (!rho_d[q]) return fail(TG_EINVAL, "NULL density pointer");
    tg_grid* g = b->grids[i];
    g->desc.ext0 = rho_d[q];
    g->desc.rho_min = rho_min[q];
    g->p = p;
    g->rho_min = rho_min[q];
  }
  b->p = p;
  int rc = batch_upload_desc(b, s);
  if (rc) return rc;
  rc = batch_set_active(b, which, s, true);
  if (rc) return rc;
  rc = k_set_density(b, s);
  if (rc) return rc;
  std::vector<int> flag(b->n, 0);
  TG_HIP(hipMemcpyAsync(flag.data(), b->flag_d, sizeof(int) * b->n, hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  bool badrho = false;
  for (int i : which) {
    b->grids[i]->density_set = !(flag[i] & 1);
    b->grids[i]->numeric_bad = (flag[i] & 2) != 0;
    badrho = badrho || (flag[i] & 1);
  }
  if (badrho) return fail(TG_EINVAL, "density outside [0, 1] or not finite");
  return TG_OK;
}

static int check_ready(Batch* b, const std::vector<int>& which, bool need_mg = false) {
  for (int i : which) {
    if (!b->grids[i]->density_set) return fail(TG_ESTATE, "set_density must be called first");
    if (need_mg && !b->grids[i]->coarse_ok)
      return fail(TG_EINVAL, "grid cannot be coarsened to a level with <= 512 free DOFs: no V-cycle");
  }
  return TG_OK;
}

// A run of FGMRES steps as a captured graph.  The steps' kernels depend only
// on the device work lists (their signature), the step range and the
// options, never on host values that change between replays (the iteration
// count and the status live on the device), so a graph is captured once per
// key and replayed on the caller's stream.  Capture runs on a private stream
// (default priority); nothing executes during capture and the timer records
// no events.
template <class F>
static int graph_run(Batch* b, F&& steps, const tg_solver_opts* o, int j0, int j1, hipStream_t s) {
  char key[192];
  std::snprintf(key, sizeof(key), "%llx|%d|%d|%d|%d|%d|%.17g|%.17g|%d", b->lists_sig, o->prec, o->cgs_passes, j0,
                j1, o->max_iters, o->tol, o->breakdown, b->grids[0]->mmax);
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    if (b->graphs.size() >= 1024) {
      for (auto& kv : b->graphs) hipGraphExecDestroy(kv.second);
      b->graphs.clear();
    }
    if (!b->cap_stream) TG_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    TG_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    timer_suspend(true);
    const int rc = steps(b->cap_stream);
    timer_suspend(false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
    it = b->graphs.emplace(key, ex).first;
  }
  TG_HIP(hipGraphLaunch(it->second, s));
  return TG_OK;
}

// Right-preconditioned FGMRES on every problem in `which` (Sec. 3.5), x0 = 0,
// rhs in slot S_F, solution in slot S_X, history in small + hist.
// Periodic true-residual checkpoints of a running FGMRES: after every
// `every` iterations, ||f - K x_k|| / ||f|| in FP64 for the iterate
// x_k = x + Z y_k of each problem that made iteration k (y_k: the least
// squares over the columns so far).  x is saved in S_T and restored; S_R,
// the dot scratch and y are free between steps and rewritten later, and the
// value goes to small[SC_TRUE] only, so the iteration is unchanged.
struct Checkpoints {
  int every = 0;
  std::vector<std::vector<std::pair<int, double>>> rec;   // per problem of the batch
};

static int checkpoint_eval(Batch* b, const std::vector<int>& act, int mmax, int jmax, int k, Checkpoints* cp,
                           hipStream_t s);
static int checkpoint(Batch* b, const std::vector<int>& act, int mmax, int jmax, int k, Checkpoints* cp,
                      hipStream_t s) {
  int rc;
  // a problem that stopped at this very step is still checked: the step
  // gate is off while the checkpoint runs
  const bool was_gated = b->gated;
  if (was_gated) {
    b->gated = false;
    if ((rc = batch_upload_desc(b, s))) return rc;
  }
  rc = checkpoint_eval(b, act, mmax, jmax, k, cp, s);
  if (was_gated) {
    b->gated = true;
    const int r2 = batch_upload_desc(b, s);
    if (!rc) rc = r2;
  }
  return rc;
}

static int checkpoint_eval(Batch* b, const std::vector<int>& act, int mmax, int jmax, int k, Checkpoints* cp,
                           hipStream_t s) {
  int rc;
  if ((rc = batch_set_active(b, act, s))) return rc;
  if ((rc = k_copy0(b, S_X, S_T, s))) return rc;
  if ((rc = k_lsq_update(b, mmax, jmax, s))) return rc;
  if ((rc = k_residual64(b, S_F, S_X, S_R, s))) return rc;
  if ((rc = k_multidot(b, 0, 0, S_R, 1, s))) return rc;
  if ((rc = k_reduce(b, 1, 2, 0, -1, s))) return rc;
  if ((rc = k_multidot(b, 0, 0, S_F, 1, s))) return rc;
  if ((rc = k_reduce(b, 1, 2, 1, -1, s))) return rc;
  if ((rc = k_true_eta(b, s, false))) return rc;
  if ((rc = k_copy0(b, S_T, S_X, s))) return rc;
  std::vector<double> v(act.size());
  for (size_t i = 0; i < act.size(); ++i) {
    const tg_grid* g = b->grids[act[i]];
    TG_HIP(hipMemcpyAsync(&v[i], g->desc.small + g->sl.scal + SC_TRUE, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  TG_HIP(hipStreamSynchronize(s));
  for (size_t i = 0; i < act.size(); ++i) cp->rec[act[i]].push_back({k, v[i]});
  return TG_OK;
}

// Turns the step gate off again on every way out of fgmres_batch.
struct GateOff {
  Batch* b;
  hipStream_t s;
  ~GateOff() {
    if (b->gated) {
      b->gated = false;
      batch_upload_desc(b, s);
    }
  }
};

static int fgmres_batch_impl(Batch* b, const std::vector<int>& which, const tg_solver_opts* o, hipStream_t s,
                             Checkpoints* cp);

int fgmres_batch(Batch* b, const std::vector<int>& which, const tg_solver_opts* o, hipStream_t s,
                 Checkpoints* cp = nullptr) {
  GateOff off{b, s};
  return fgmres_batch_impl(b, which, o, s, cp);
}

static int fgmres_batch_impl(Batch* b, const std::vector<int>& which, const tg_solver_opts* o, hipStream_t s,
                             Checkpoints* cp) {
  const int m = o->restart, cap = o->max_iters;
  const int mmax = b->grids[0]->mmax;
  if (m < 1 || m > mmax) return fail(TG_EINVAL, "restart must be in [1, bound max_restart]");
  if (cap < 0 || cap > TG_HIST_CAP - 1) return fail(TG_EINVAL, "max_iters out of range");
  if (o->cgs_passes < 1 || o->cgs_passes > 3) return fail(TG_EINVAL, "cgs_passes must be 1, 2 or 3");
  const bool delayed = o->cgs_passes == 2;
  if (o->prec < TG_F64 || o->prec > TG_BF16X3MFMA)
    return fail(TG_EINVAL, "unknown preconditioner precision");
  const double tol = o->tol, brk = o->breakdown;
  if (cp && o->graphs) return fail(TG_EINVAL, "checkpoints are not taken under graph replay");
  if (o->sync_every < 1) return fail(TG_EINVAL, "sync_every must be >= 1");
  const int K = (cp && cp->every > 0) ? 1 : o->sync_every;
  if (cp) cp->rec.assign(b->n, {});
  int rc = check_ready(b, which, true);
  if (rc) return rc;
  rc = batch_set_active(b, which, s);
  if (rc) return rc;
  if ((rc = k_init_small(b, s))) return rc;
  if ((rc = k_fill0(b, S_X, 0.0, s))) return rc;
  // cycle-start residual: the delayed form keeps it unnormalized in V_0
  const int SR = delayed ? slot_V(0) : S_R;
  if ((rc = k_copy0(b, S_F, SR, s))) return rc;
  std::vector<int> running = which;
  int k = 0;
  while (true) {
    if ((rc = batch_set_active(b, running, s))) return rc;
    if (k > 0 && (rc = k_residual64(b, S_F, S_X, SR, s))) return rc;
    if ((rc = k_multidot(b, 0, 0, SR, 1, s))) return rc;
    if ((rc = k_reduce(b, 1, 2, 0, -1, s))) return rc;
    if ((rc = k_cycle_start(b, k, cap, tol, s))) return rc;
    if ((rc = batch_read_status(b, s))) return rc;
    if (!b->gated) {
      // the status gather now holds every running problem's state: from here
      // on the step kernels skip the problems that stop
      b->gated = true;
      if ((rc = batch_upload_desc(b, s))) return rc;
    }
    std::vector<int> nr;
    for (int i : running)
      if (b->sc_h[i] == TG_RUNNING) nr.push_back(i);
    running.swap(nr);
    if (running.empty()) break;
    if ((rc = batch_set_active(b, running, s))) return rc;
    if (!delayed && (rc = k_scale_to(b, S_R, slot_V(0), SC_INV, s))) return rc;
    const std::vector<int> members = running;
    int jmax = 0;
    // Runs of up to K Arnoldi steps between host reads of the status: a
    // problem that stops inside a run is skipped on the device by the rest
    // of it (the step kernels' gate), so every run leaves each problem
    // exactly as single steps would.
    for (int j0 = 0; j0 < m;) {
      const int j1 = std::min(m, j0 + K);
      const int k0 = k;
      auto one_step = [&](int j, int kk, hipStream_t st) -> int {
        int r;
        if (delayed) {
          // CGS2 with delayed reorthogonalization: V_j holds q~_j (projected
          // once, first-pass norm rho_j in SC_RHO); z_j = M^-1 (q~_j / rho_j).
          // Sweep A: dots of [V_0..V_{j-1}, q~_j] with q~_j and w = K z_j;
          // sweep B: reorthogonalized q_j into V_j and q~_{j+1} into V_{j+1}.
          if ((r = k_vcycle(b, o->prec, 0, slot_V(j), nullptr, 0, slot_Z(mmax, j), nullptr, st, SC_INV)))
            return r;
          if ((r = k_apply(b, TG_F64, slot_Z(mmax, j), nullptr, S_W, nullptr, st))) return r;
          // (each sweep is followed by one per-problem launch that sums its
          // chunk partials and runs that part's scalar work)
          if ((r = k_dots2(b, slot_V(0), j, slot_V(j), S_W, st))) return r;
          return k_update2(b, slot_V(0), j, slot_V(j), S_W, slot_V(j + 1), cap, tol, brk, st);
        }
        if ((r = k_vcycle(b, o->prec, 0, slot_V(j), nullptr, 0, slot_Z(mmax, j), nullptr, st))) return r;
        if ((r = k_apply(b, TG_F64, slot_Z(mmax, j), nullptr, S_W, nullptr, st))) return r;
        // Classical Gram-Schmidt, each pass h = V^T w then w -= V h, in fused
        // sweeps: [dots1 (+ w.w before projection -> SC_FLAG, breakdown test)]
        // [w -= V h1; dots2] [w -= V h2; w.w]  (CGS2), or [dots1] [w -= V h1; w.w].
        if ((r = k_multidot(b, slot_V(0), j + 1, S_W, 1, st))) return r;
        if ((r = k_reduce(b, j + 2, 0, 0, j + 1, st))) return r;
        if (o->cgs_passes == 3) {
          if ((r = k_update_dots(b, slot_V(0), j + 1, S_W, 0, j + 1, 0, st))) return r;
          if ((r = k_reduce(b, j + 1, 1, 0, -1, st))) return r;
          if ((r = k_update_dots(b, slot_V(0), j + 1, S_W, 1, 0, 1, st))) return r;
        } else {
          if ((r = k_update_dots(b, slot_V(0), j + 1, S_W, 0, 0, 1, st))) return r;
        }
        if ((r = k_reduce(b, 1, 2, 0, -1, st))) return r;
        if ((r = k_arnoldi(b, j, kk, cap, tol, brk, st))) return r;
        return k_scale_to(b, S_W, slot_V(j + 1), SC_INV, st);
      };
      auto run = [&](hipStream_t st) -> int {
        for (int j = j0; j < j1; ++j) {
          const int r = one_step(j, k0 + (j - j0), st);
          if (r) return r;
        }
        return TG_OK;
      };
      if (o->graphs) {
        if ((rc = graph_run(b, run, o, j0, j1, s))) return rc;
      } else if ((rc = run(s))) {
        return rc;
      }
      k += j1 - j0;   // every problem still running made each step of the run
      jmax = j1;
      if ((rc = batch_read_status(b, s))) return rc;
      if (cp && cp->every > 0 && k % cp->every == 0 && (rc = checkpoint(b, running, mmax, jmax, k, cp, s)))
        return rc;
      std::vector<int> still;
      for (int i : running)
        if (b->sc_h[i] == TG_RUNNING) still.push_back(i);
      if (still.empty() || j1 == m) break;
      if (still.size() != running.size()) {
        running.swap(still);
        if ((rc = batch_set_active(b, running, s))) return rc;
      }
      j0 = j1;
    }
    // end of cycle: y = R^-1 g, x += Z y for every problem of this cycle
    if ((rc = batch_set_active(b, members, s))) return rc;
    if ((rc = k_lsq_update(b, mmax, jmax, s))) return rc;
    if ((rc = batch_read_status(b, s))) return rc;
    running.clear();
    for (int i : members)
      if (b->sc_h[i] == TG_RUNNING) running.push_back(i);
    if (running.empty()) break;
  }
  TG_HIP(hipStreamSynchronize(s));
  return TG_OK;
}

// eta = ||f - K x|| / ||f|| (FP64, free DOFs) from slots S_F, S_X; writes sc_h.
int true_residual_batch(Batch* b, const std::vector<int>& which, hipStream_t s) {
  int rc = batch_set_active(b, which, s);
  if (rc) return rc;
  if ((rc = k_residual64(b, S_F, S_X, S_R, s))) return rc;
  if ((rc = k_multidot(b, 0, 0, S_R, 1, s))) return rc;
  if ((rc = k_reduce(b, 1, 2, 0, -1, s))) return rc;
  if ((rc = k_multidot(b, 0, 0, S_F, 1, s))) return rc;
  if ((rc = k_reduce(b, 1, 2, 1, -1, s))) return rc;
  if ((rc = k_true_eta(b, s))) return rc;
  return batch_read_status(b, s);
}

// Copy external per-problem vectors into / out of level-0 slots.
int copy_in_batch(Batch* b, const std::vector<int>& which, const double* const* src, int slot,
                  hipStream_t s) {
  for (int q = 0; q < (int)which.size(); ++q) b->grids[which[q]]->desc.ext0 = src[q];
  int rc = batch_upload_desc(b, s);
  if (rc) return rc;
  if ((rc = batch_set_active(b, which, s))) return rc;
  return k_copy_ext(b, 0, slot, s);
}
int copy_out_batch(Batch* b, const std::vector<int>& which, double* const* dst, int slot,
                   hipStream_t s) {
  for (int q = 0; q < (int)which.size(); ++q) b->grids[which[q]]->desc.ext1 = dst[q];
  int rc = batch_upload_desc(b, s);
  if (rc) return rc;
  if ((rc = batch_set_active(b, which, s))) return rc;
  return k_copy_ext(b, 1, slot, s);
}

struct ScalRead {
  double v[32];
};
static int read_scal(Batch* b, int i, ScalRead& r, hipStream_t s) {
  tg_grid* g = b->grids[i];
  TG_HIP(hipMemcpyAsync(r.v, g->desc.small + g->sl.scal, sizeof(r.v), hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  return TG_OK;
}
static int read_hist(Batch* b, int i, int count, double* h, hipStream_t s) {
  tg_grid* g = b->grids[i];
  TG_HIP(hipMemcpyAsync(h, g->desc.small + g->sl.hist, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  return TG_OK;
}

static void fill_result(const ScalRead& r, tg_solve_result* res) {
  res->iterations = (int)r.v[SC_ITERS];
  res->outcome = (int)r.v[SC_STATUS];
  res->proj_eta = r.v[SC_EST];
  res->true_eta = -1.0;
}

// ---------------------------------------------------------------------------
// Probe features (Sec. 3.4) from a probe history.
void probe_feats(const double* hist, int kstop, double* r50, double* r100) {
  *r50 = hist[std::min(50, kstop)];
  *r100 = hist[std::min(100, kstop)];
}

int rule_fires(const tg_policy* pol, double r50, double r100) {
  return (r50 >= pol->t_high) || (r100 >= pol->t_plateau && r100 / r50 >= pol->t_ratio);
}

// Alg. floor_policy for every problem of the batch.
int select_floor_batch(Batch* b, const double* const* rho_d, const double* const* f_d,
                       const tg_policy* pol, double* const* u_d, tg_policy_result* out,
                       hipStream_t s) {
  if (!pol || pol->n_rungs < 1 || pol->n_rungs > TG_MAX_RUNGS) return fail(TG_EINVAL, "bad policy rungs");
  for (int r = 0; r < pol->n_rungs; ++r)
    if (!(pol->rungs[r] > 0 && pol->rungs[r] <= 1)) return fail(TG_EINVAL, "rungs must be in (0, 1]");
  const int n = b->n;
  const std::vector<int> all = all_of(b);
  std::memset(out, 0, sizeof(tg_policy_result) * n);
  int rc;
  // ---- probe at the original floor
  std::vector<double> r0(n, pol->rungs[0]);
  if ((rc = set_density_batch(b, all, rho_d, pol->p, r0.data(), s))) return rc;
  if ((rc = copy_in_batch(b, all, f_d, S_F, s))) return rc;
  tg_solver_opts po = pol->solve;
  po.restart = pol->probe_restart;
  po.max_iters = pol->probe_iters;
  if ((rc = fgmres_batch(b, all, &po, s))) return rc;
  std::vector<int> k0(n, 0);
  std::vector<std::array<float, 8>> feats(n);
  for (int i = 0; i < n; ++i) {
    ScalRead sr;
    if ((rc = read_scal(b, i, sr, s))) return rc;
    const int kstop = (int)sr.v[SC_ITERS];
    std::vector<double> h(kstop + 1);
    if ((rc = read_hist(b, i, kstop + 1, h.data(), s))) return rc;
    probe_feats(h.data(), kstop, &out[i].r50, &out[i].r100);
    out[i].probe_iters = kstop;
    out[i].iters_probe = kstop;
    k0[i] = rule_fires(pol, out[i].r50, out[i].r100) ? std::min(1, pol->n_rungs - 1) : 0;
    feats[i][0] = (float)std::log10(std::max(out[i].r50, 1e-300));
    feats[i][1] = (float)std::log10(std::max(out[i].r100, 1e-300));
  }
  const bool use_mlp = pol->selector == TG_SELECT_MLP && pol->mlp;
  if (use_mlp || pol->want_features)
    if ((rc = density_features(b, all, rho_d, pol->p, pol->rungs[0], feats, s))) return rc;
  if (use_mlp) {
    std::vector<int> pred;
    if ((rc = mlp_select(pol->mlp, feats, pred, s))) return rc;
    for (int i = 0; i < n; ++i) k0[i] = std::min(std::max(pred[i], 0), pol->n_rungs - 1);
  } else if (pol->selector == TG_SELECT_FIXED) {
    for (int i = 0; i < n; ++i) k0[i] = std::min(std::max(pol->fixed_rung, 0), pol->n_rungs - 1);
  }
  for (int i = 0; i < n; ++i) {
    out[i].k0 = k0[i];
    out[i].rung = -1;
    out[i].floor = -1.0;
    for (int q = 0; q < 8; ++q) out[i].features[q] = feats[i][q];
  }
  // ---- guarded ladder: independent solve, recomputed FP64 residual, climb
  std::vector<int> rung = k0;
  std::vector<int> pending = all;
  while (!pending.empty()) {
    std::vector<double> fl(pending.size());
    std::vector<const double*> rp(pending.size()), fp(pending.size());
    for (size_t q = 0; q < pending.size(); ++q) {
      fl[q] = pol->rungs[rung[pending[q]]];
      rp[q] = rho_d[pending[q]];
      fp[q] = f_d[pending[q]];
    }
    if ((rc = set_density_batch(b, pending, rp.data(), pol->p, fl.data(), s))) return rc;
    if ((rc = copy_in_batch(b, pending, fp.data(), S_F, s))) return rc;
    if ((rc = fgmres_batch(b, pending, &pol->solve, s))) return rc;
    if ((rc = true_residual_batch(b, pending, s))) return rc;
    std::vector<int> next;
    for (int i : pending) {
      ScalRead sr;
      if ((rc = read_scal(b, i, sr, s))) return rc;
      tg_policy_result& R = out[i];
      auto& A = R.attempts[R.n_attempts++];
      A.rung = rung[i];
      A.floor = pol->rungs[rung[i]];
      A.iterations = (int)sr.v[SC_ITERS];
      A.outcome = (int)sr.v[SC_STATUS];
      A.proj_eta = sr.v[SC_EST];
      A.true_eta = sr.v[SC_TRUE];
      A.accepted = (A.true_eta <= pol->tau) && std::isfinite(A.true_eta);
      if (A.accepted) {
        R.rung = rung[i];
        R.floor = A.floor;
        R.iters_selected = A.iterations;
      } else {
        R.iters_rejected += A.iterations;
        if (rung[i] + 1 < pol->n_rungs) {
          rung[i] += 1;
          next.push_back(i);
        }
      }
    }
    // accepted solutions out
    std::vector<int> acc;
    std::vector<double*> dst;
    for (int i : pending)
      if (out[i].rung >= 0 && out[i].attempts[out[i].n_attempts - 1].accepted) {
        acc.push_back(i);
        dst.push_back(u_d[i]);
      }
    if (!acc.empty() && (rc = copy_out_batch(b, acc, dst.data(), S_X, s))) return rc;
    pending.swap(next);
  }
  // no admissible floor: zero solution
  std::vector<int> none;
  std::vector<double*> dn;
  for (int i = 0; i < n; ++i)
    if (out[i].rung < 0) {
      none.push_back(i);
      dn.push_back(u_d[i]);
    }
  if (!none.empty()) {
    if ((rc = batch_set_active(b, none, s))) return rc;
    if ((rc = k_fill0(b, S_T, 0.0, s))) return rc;
    if ((rc = copy_out_batch(b, none, dn.data(), S_T, s))) return rc;
  }
  TG_HIP(hipStreamSynchronize(s));
  return TG_OK;
}

}  // namespace tg

// ===========================================================================
using namespace tg;

extern "C" {

int tg_set_density(tg_grid* g, const double* rho_d, double p, double rho_min, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  const int rc = set_density_batch(g->self, {0}, &rho_d, p, &rho_min, S(stream));
  if (rc) return rc;
  if (g->numeric_bad) return fail(TG_ENUMERIC, "coarsest-level Cholesky met a non-positive pivot");
  return TG_OK;
}

int tg_apply_K(const tg_grid* gc, const void* u_d, void* y_d, int prec, void* stream) {
  tg_grid* g = const_cast<tg_grid*>(gc);
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!u_d || !y_d) return fail(TG_EINVAL, "NULL vector");
  if (prec < TG_F64 || prec > TG_BF16X3MFMA) return fail(TG_EINVAL, "unknown precision");
  int rc = check_ready(g->self, {0});
  if (rc) return rc;
  if ((rc = batch_set_active(g->self, {0}, S(stream)))) return rc;
  return k_apply(g->self, prec, -1, u_d, -1, y_d, S(stream));
}

int tg_vcycle(tg_grid* g, const void* r_d, void* z_d, int prec, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!r_d || !z_d) return fail(TG_EINVAL, "NULL vector");
  if (prec < TG_F64 || prec > TG_BF16X3MFMA) return fail(TG_EINVAL, "unknown precision");
  int rc = check_ready(g->self, {0}, true);
  if (rc) return rc;
  if ((rc = batch_set_active(g->self, {0}, S(stream)))) return rc;
  const int f32 = prec != TG_F64;
  return k_vcycle(g->self, prec, f32, -1, r_d, f32, -1, z_d, S(stream));
}

int tg_fgmres_solve(tg_grid* g, const double* f_d, double* u_d, const tg_solver_opts* o,
                    tg_solve_result* res, double* hist_h, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!f_d || !u_d || !o || !res) return fail(TG_EINVAL, "NULL argument");
  Batch* b = g->self;
  hipStream_t s = S(stream);
  int rc = check_ready(b, {0});
  if (rc) return rc;
  if ((rc = copy_in_batch(b, {0}, &f_d, S_F, s))) return rc;
  if ((rc = fgmres_batch(b, {0}, o, s))) return rc;
  if ((rc = copy_out_batch(b, {0}, &u_d, S_X, s))) return rc;
  ScalRead sr;
  if ((rc = read_scal(b, 0, sr, s))) return rc;
  fill_result(sr, res);
  if (hist_h && (rc = read_hist(b, 0, res->iterations + 1, hist_h, s))) return rc;
  return TG_OK;
}

int tg_true_residual(const tg_grid* gc, const double* f_d, const double* u_d, double* eta_h, void* stream) {
  tg_grid* g = const_cast<tg_grid*>(gc);
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!f_d || !u_d || !eta_h) return fail(TG_EINVAL, "NULL argument");
  Batch* b = g->self;
  hipStream_t s = S(stream);
  int rc = check_ready(b, {0});
  if (rc) return rc;
  if ((rc = copy_in_batch(b, {0}, &f_d, S_F, s))) return rc;
  if ((rc = copy_in_batch(b, {0}, &u_d, S_X, s))) return rc;
  if ((rc = true_residual_batch(b, {0}, s))) return rc;
  *eta_h = b->sc_h[0];
  return TG_OK;
}

int tg_probe_features(tg_grid* g, const double* f_d, const tg_solver_opts* o, int iters,
                      double* r50_h, double* r100_h, int* k_stop_h, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!f_d || !o || !r50_h || !r100_h) return fail(TG_EINVAL, "NULL argument");
  Batch* b = g->self;
  hipStream_t s = S(stream);
  int rc = check_ready(b, {0});
  if (rc) return rc;
  tg_solver_opts po = *o;
  po.max_iters = iters;
  if ((rc = copy_in_batch(b, {0}, &f_d, S_F, s))) return rc;
  if ((rc = fgmres_batch(b, {0}, &po, s))) return rc;
  ScalRead sr;
  if ((rc = read_scal(b, 0, sr, s))) return rc;
  const int kstop = (int)sr.v[SC_ITERS];
  std::vector<double> h(kstop + 1);
  if ((rc = read_hist(b, 0, kstop + 1, h.data(), s))) return rc;
  probe_feats(h.data(), kstop, r50_h, r100_h);
  if (k_stop_h) *k_stop_h = kstop;
  return TG_OK;
}

int tg_probe_checkpoints(tg_grid* g, const double* f_d, const tg_solver_opts* o, int iters, int every, int cap,
                         int* k_h, double* proj_h, double* true_h, int* n_h, int* k_stop_h, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!f_d || !o || !k_h || !proj_h || !true_h || !n_h) return fail(TG_EINVAL, "NULL argument");
  if (every < 1 || cap < 0) return fail(TG_EINVAL, "need every >= 1 and cap >= 0");
  Batch* b = g->self;
  hipStream_t s = S(stream);
  int rc = check_ready(b, {0});
  if (rc) return rc;
  tg_solver_opts po = *o;
  po.max_iters = iters;
  Checkpoints cp;
  cp.every = every;
  if ((rc = copy_in_batch(b, {0}, &f_d, S_F, s))) return rc;
  if ((rc = fgmres_batch(b, {0}, &po, s, &cp))) return rc;
  ScalRead sr;
  if ((rc = read_scal(b, 0, sr, s))) return rc;
  const int kstop = (int)sr.v[SC_ITERS];
  std::vector<double> h(kstop + 1);
  if ((rc = read_hist(b, 0, kstop + 1, h.data(), s))) return rc;
  const auto& r = cp.rec[0];
  const int n = std::min<int>(cap, (int)r.size());
  for (int i = 0; i < n; ++i) {
    k_h[i] = r[i].first;
    true_h[i] = r[i].second;
    proj_h[i] = r[i].first <= kstop ? h[r[i].first] : -1.0;
  }
  *n_h = n;
  if (k_stop_h) *k_stop_h = kstop;
  return TG_OK;
}

void tg_default_policy(tg_policy* pol) {
  if (!pol) return;
  std::memset(pol, 0, sizeof(*pol));
  pol->n_rungs = 4;
  pol->rungs[0] = 1e-9;
  pol->rungs[1] = 1e-6;
  pol->rungs[2] = 1e-4;
  pol->rungs[3] = 1e-3;
  pol->p = 3.0;
  pol->tau = 1e-6;
  pol->probe_iters = 100;
  pol->probe_restart = 100;
  pol->t_high = 1e-2;
  pol->t_plateau = 1e-4;
  pol->t_ratio = 0.6;
  pol->selector = TG_SELECT_RULE;
  pol->fixed_rung = 0;
  pol->mlp = nullptr;
  tg_default_solver_opts(&pol->solve);
  pol->want_features = 0;
}

int tg_select_floor(tg_grid* g, const double* rho_d, const double* f_d, const tg_policy* pol,
                    double* u_d, tg_policy_result* out, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!rho_d || !f_d || !pol || !u_d || !out) return fail(TG_EINVAL, "NULL argument");
  return select_floor_batch(g->self, &rho_d, &f_d, pol, &u_d, out, S(stream));
}

// ---- batches ----------------------------------------------------------------
struct tg_batch {
  tg::Batch b;
};

int tg_batch_create(int n, tg_grid* const* grids, tg_batch** out) {
  if (!out || !grids) return fail(TG_EINVAL, "NULL argument");
  *out = nullptr;
  tg_batch* tb = new tg_batch();
  int rc = batch_init(&tb->b, n, grids);
  if (rc) {
    delete tb;
    return rc;
  }
  *out = tb;
  return TG_OK;
}
void tg_batch_destroy(tg_batch* b) { delete b; }
int tg_batch_workspace_bytes(const tg_batch* b, size_t* bytes) {
  if (!b || !bytes) return fail(TG_EINVAL, "NULL argument");
  *bytes = batch_ws_bytes_for(b->b.grids);
  return TG_OK;
}
int tg_batch_bind_workspace(tg_batch* b, void* ws_d, size_t bytes) {
  if (!b) return fail(TG_EINVAL, "NULL batch");
  return batch_bind(&b->b, ws_d, bytes);
}
int tg_batch_set_density(tg_batch* tb, const double* const* rho_d, double p, const double* rho_min_h,
                         void* stream) {
  if (!tb || !rho_d || !rho_min_h) return fail(TG_EINVAL, "NULL argument");
  if (!tb->b.ws) return fail(TG_EWORKSPACE, "batch workspace not bound");
  return set_density_batch(&tb->b, all_of(&tb->b), rho_d, p, rho_min_h, S(stream));
}
int tg_batch_solve(tg_batch* tb, const double* const* f_d, double* const* u_d, const tg_solver_opts* o,
                   tg_solve_result* res, void* stream) {
  if (!tb || !f_d || !u_d || !o || !res) return fail(TG_EINVAL, "NULL argument");
  if (!tb->b.ws) return fail(TG_EWORKSPACE, "batch workspace not bound");
  Batch* b = &tb->b;
  hipStream_t s = S(stream);
  const std::vector<int> all = all_of(b);
  int rc = check_ready(b, all);
  if (rc) return rc;
  if ((rc = copy_in_batch(b, all, f_d, S_F, s))) return rc;
  if ((rc = fgmres_batch(b, all, o, s))) return rc;
  if ((rc = true_residual_batch(b, all, s))) return rc;
  for (int i = 0; i < b->n; ++i) {
    ScalRead sr;
    if ((rc = read_scal(b, i, sr, s))) return rc;
    fill_result(sr, &res[i]);
    res[i].true_eta = sr.v[SC_TRUE];
  }
  return copy_out_batch(b, all, u_d, S_X, s);
}
int tg_batch_tile_heights(const tg_batch* tb, int i, int* zc_out) {
  if (!tb || !zc_out) return fail(TG_EINVAL, "NULL argument");
  if (i < 0 || i >= tb->b.n) return fail(TG_EINVAL, "problem index out of range");
  const tg_grid* g = tb->b.grids[i];
  for (int l = 0; l < TG_MAXLEV; ++l)
    zc_out[l] = (l < g->nlev) ? zm_height(g->lv[l].ez + 1, batch_zc(&tb->b, i, l)) : 0;
  return TG_OK;
}
int tg_batch_history(const tg_batch* tb, int i, int count, double* hist_h, void* stream) {
  if (!tb || !hist_h) return fail(TG_EINVAL, "NULL argument");
  if (!tb->b.ws) return fail(TG_EWORKSPACE, "batch workspace not bound");
  if (i < 0 || i >= tb->b.n) return fail(TG_EINVAL, "problem index out of range");
  if (count < 0 || count > TG_HIST_CAP) return fail(TG_EINVAL, "count out of range");
  if (count == 0) return TG_OK;
  return read_hist(const_cast<Batch*>(&tb->b), i, count, hist_h, S(stream));
}
int tg_batch_autotune(tg_batch* tb, int prec, int force, int* zc_out, double* us_out, void* stream) {
  if (!tb) return fail(TG_EINVAL, "NULL batch");
  if (!tb->b.ws) return fail(TG_EWORKSPACE, "batch workspace not bound");
  const int rc = autotune_batch(&tb->b, prec, S(stream), us_out, force != 0);
  if (rc) return rc;
  if (zc_out)
    for (int l = 0; l < TG_MAXLEV; ++l) zc_out[l] = tb->b.zc[l];
  return TG_OK;
}
int tg_autotune(tg_grid* g, int prec, int force, int* zc_out, double* us_out, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  const int rc = autotune_batch(g->self, prec, S(stream), us_out, force != 0);
  if (rc) return rc;
  if (zc_out)
    for (int l = 0; l < TG_MAXLEV; ++l) zc_out[l] = g->self->zc[l];
  return TG_OK;
}

int tg_batch_select_floor(tg_batch* tb, const double* const* rho_d, const double* const* f_d,
                          const tg_policy* pol, double* const* u_d, tg_policy_result* out,
                          void* stream) {
  if (!tb || !rho_d || !f_d || !pol || !u_d || !out) return fail(TG_EINVAL, "NULL argument");
  if (!tb->b.ws) return fail(TG_EWORKSPACE, "batch workspace not bound");
  return select_floor_batch(&tb->b, rho_d, f_d, pol, u_d, out, S(stream));
}

}  // extern "C"
