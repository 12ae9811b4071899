// The optimizer around the guarded state solve: the minimum-compliance loop
// of Sec. 3.1 (Eq. to_problem) with the linear-hat density filter, the
// smoothed Heaviside projection (Eq. projection), the optimality-criteria
// update with a move limit and a bisection on the volume multiplier, and the
// two-stage continuation of Tab. trajectory-settings; the floor is chosen at
// every outer iteration by the guarded policy (Alg. floor_policy), optionally
// reusing the previous decision until the guard rejects it (the cost
// reduction Sec. 5.2 names as untested), or fixed without acceptance test
// (the controls of Sec. 4.1.2).
//
// Filter, projection and OC kernels are elementwise or small stencils over
// the element grid (x fastest); every sum runs in a fixed order.  The
// bisection and the loop run on the host around them: each step needs one
// scalar (the volume, the largest change) back.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "tg_internal.h"

namespace tg {
namespace {

constexpr int TO_BLOCK = 256;
constexpr int TO_MAX_R = 3;       // stencil half-width: r_min < 4

__device__ __forceinline__ void elem_ijk(long long e, int nx, int ny, int& i, int& j, int& k) {
  i = (int)(e % nx);
  const long long r = e / nx;
  j = (int)(r % ny);
  k = (int)(r / ny);
}

// sum_j w_ej a_j (b_j) / (sum_j w_ej) over the in-grid neighbours j of e,
// w = r - |d| > 0, |d_i| <= R; the offset order is fixed.
__device__ __forceinline__ void hat_sums(int i, int j, int k, int nx, int ny, int nz, int R, double r,
                                         const double* a, double& s, double& W) {
  s = 0.0;
  W = 0.0;
  for (int dz = -R; dz <= R; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const double w = r - sqrt((double)(dx * dx + dy * dy + dz * dz));
        const int ii = i + dx, jj = j + dy, kk = k + dz;
        if (w <= 0 || ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
        W += w;
        if (a) s += w * a[ii + (long long)nx * (jj + (long long)ny * kk)];
      }
}

// xt = H x (and, if beta > 0, xbar = project(xt), dxbar its derivative).
__global__ __launch_bounds__(TO_BLOCK) void k_filter(const double* __restrict__ x, int nx, int ny, int nz,
                                                     int R, double r, double beta, double eta,
                                                     double* __restrict__ xt, double* __restrict__ xbar,
                                                     double* __restrict__ dxbar) {
  const long long n = (long long)nx * ny * nz;
  for (long long e = (long long)blockIdx.x * TO_BLOCK + threadIdx.x; e < n; e += (long long)gridDim.x * TO_BLOCK) {
    int i, j, k;
    elem_ijk(e, nx, ny, i, j, k);
    double s, W;
    hat_sums(i, j, k, nx, ny, nz, R, r, x, s, W);
    const double v = s / W;
    if (xt) xt[e] = v;
    if (xbar) {
      const double den = tanh(beta * eta) + tanh(beta * (1.0 - eta));
      const double th = tanh(beta * (v - eta));
      xbar[e] = fmin(1.0, fmax(0.0, (tanh(beta * eta) + th) / den));   // rounding stays in [0, 1]
      if (dxbar) dxbar[e] = beta * (1.0 - th * th) / den;
    }
  }
}

// y_j = sum_e w_ej a_e b_e / W_e (b may be NULL: 1), W_e recomputed for each
// neighbour e (the stencil is symmetric, so e runs over j's own stencil).
__global__ __launch_bounds__(TO_BLOCK) void k_filter_adj(const double* __restrict__ a,
                                                         const double* __restrict__ b, int nx, int ny,
                                                         int nz, int R, double r, double* __restrict__ y) {
  const long long n = (long long)nx * ny * nz;
  for (long long e = (long long)blockIdx.x * TO_BLOCK + threadIdx.x; e < n; e += (long long)gridDim.x * TO_BLOCK) {
    int i, j, k;
    elem_ijk(e, nx, ny, i, j, k);
    double acc = 0.0;
    for (int dz = -R; dz <= R; ++dz)
      for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
          const double w = r - sqrt((double)(dx * dx + dy * dy + dz * dz));
          const int ii = i + dx, jj = j + dy, kk = k + dz;
          if (w <= 0 || ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
          const long long q = ii + (long long)nx * (jj + (long long)ny * kk);
          double s, W;
          hat_sums(ii, jj, kk, nx, ny, nz, R, r, nullptr, s, W);
          acc += w * (b ? a[q] * b[q] : a[q]) / W;
        }
    y[e] = acc;
  }
}

// x_new = clip(x sqrt(max(0, -dc) / (lam dv)), max(0, x - move), min(1, x + move))
__global__ __launch_bounds__(TO_BLOCK) void k_oc(const double* __restrict__ x, const double* __restrict__ dc,
                                                 const double* __restrict__ dv, long long n, double lam,
                                                 double move, double* __restrict__ xn) {
  for (long long e = (long long)blockIdx.x * TO_BLOCK + threadIdx.x; e < n; e += (long long)gridDim.x * TO_BLOCK) {
    const double ratio = fmax(0.0, -dc[e]) / fmax(dv[e], 1e-300);
    const double v = x[e] * sqrt(ratio / lam);
    xn[e] = fmin(fmin(1.0, x[e] + move), fmax(fmax(0.0, x[e] - move), v));
  }
}

// Per-block partials of sum_e project(H x)_e (mode 0) or max_e |a_e - b_e|
// (mode 1), fixed order.
__global__ __launch_bounds__(TO_BLOCK) void k_to_reduce(const double* __restrict__ x, const double* __restrict__ b,
                                                        int nx, int ny, int nz, int R, double r, double beta,
                                                        double eta, int mode, double* __restrict__ part) {
  __shared__ double red[TO_BLOCK / 64];
  const long long n = (long long)nx * ny * nz;
  double acc = 0.0;
  const double den = tanh(beta * eta) + tanh(beta * (1.0 - eta));
  for (long long e = (long long)blockIdx.x * TO_BLOCK + threadIdx.x; e < n; e += (long long)gridDim.x * TO_BLOCK) {
    if (mode == 0) {
      int i, j, k;
      elem_ijk(e, nx, ny, i, j, k);
      double s, W;
      hat_sums(i, j, k, nx, ny, nz, R, r, x, s, W);
      acc += (tanh(beta * eta) + tanh(beta * (s / W - eta))) / den;
    } else {
      acc = fmax(acc, fabs(x[e] - b[e]));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(acc, off, 64);
    acc = mode == 0 ? acc + o : fmax(acc, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = red[0];
    for (int w = 1; w < TO_BLOCK / 64; ++w) s = mode == 0 ? s + red[w] : fmax(s, red[w]);
    part[blockIdx.x] = s;
  }
}

int stencil_R(double r_min) { return (int)std::floor(r_min); }

int nblocks(long long n) { return (int)std::max<long long>(1, std::min<long long>(1024, (n + TO_BLOCK - 1) / TO_BLOCK)); }

long long n_elem(const tg_grid* g) { return (long long)g->nx * g->ny * g->nz; }

int check_grid(const tg_grid* g) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  return TG_OK;
}

int check_r(double r_min) {
  if (!(r_min > 0) || !(r_min < TO_MAX_R + 1)) return fail(TG_EINVAL, "need 0 < r_min < 4");
  return TG_OK;
}

// sum (mode 0) or max (mode 1) through the grid's partial-sum scratch
int reduce_host(const tg_grid* g, const double* x, const double* b, double r, double beta, double eta, int mode,
                hipStream_t s, double* out) {
  const long long n = n_elem(g);
  const int nb = nblocks(n);
  if ((long long)nb > (long long)TG_PART_W * g->lv[0].n_chunks) return fail(TG_EINVAL, "partial buffer too small");
  if (mode == 1 && !b) return fail(TG_EINVAL, "max-change reduction needs two vectors");
  k_to_reduce<<<nb, TO_BLOCK, 0, s>>>(x, b, g->nx, g->ny, g->nz, stencil_R(r), r, beta, eta, mode, g->desc.part);
  TG_HIP(hipGetLastError());
  std::vector<double> h(nb);
  TG_HIP(hipMemcpyAsync(h.data(), g->desc.part, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  double acc = h[0];
  for (int i = 1; i < nb; ++i) acc = mode == 0 ? acc + h[i] : std::max(acc, h[i]);
  *out = acc;
  return TG_OK;
}

int oc_update(const tg_grid* g, const double* x, const double* dc, const double* dv, double volfrac, double move,
              double r, double beta, double eta, double* xn, double* lam_out, hipStream_t s) {
  const long long n = n_elem(g);
  const double target = volfrac * (double)n;
  double l1 = 0.0, l2 = 1e9, lm = 0.5e9;
  for (int it = 0; it < 200 && (l2 - l1) / (l1 + l2) > 1e-9; ++it) {
    lm = 0.5 * (l1 + l2);
    k_oc<<<nblocks(n), TO_BLOCK, 0, s>>>(x, dc, dv, n, lm, move, xn);
    TG_HIP(hipGetLastError());
    double vol = 0.0;
    const int rc = reduce_host(g, xn, nullptr, r, beta, eta, 0, s, &vol);
    if (rc) return rc;
    if (vol > target)
      l1 = lm;
    else
      l2 = lm;
  }
  if (lam_out) *lam_out = lm;
  return TG_OK;
}

}  // namespace
}  // namespace tg

using namespace tg;

extern "C" {

int tg_density_filter(const tg_grid* g, const double* x_d, double r_min, double* xt_d, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_r(r_min))) return rc;
  if (!x_d || !xt_d) return fail(TG_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  k_filter<<<nblocks(n_elem(g)), TO_BLOCK, 0, s>>>(x_d, g->nx, g->ny, g->nz, stencil_R(r_min), r_min, 0.0, 0.5,
                                                     xt_d, nullptr, nullptr);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int tg_density_filter_adjoint(const tg_grid* g, const double* a_d, const double* b_d, double r_min, double* y_d,
                              void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_r(r_min))) return rc;
  if (!a_d || !y_d) return fail(TG_EINVAL, "NULL argument");
  if (a_d == y_d || b_d == y_d) return fail(TG_EINVAL, "output must not alias an input");
  hipStream_t s = (hipStream_t)stream;
  k_filter_adj<<<nblocks(n_elem(g)), TO_BLOCK, 0, s>>>(a_d, b_d, g->nx, g->ny, g->nz, stencil_R(r_min), r_min, y_d);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int tg_filter_project(const tg_grid* g, const double* x_d, double r_min, double beta, double eta, double* xt_d,
                      double* xbar_d, double* dxbar_d, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_r(r_min))) return rc;
  if (!x_d || !xbar_d) return fail(TG_EINVAL, "NULL argument");
  if (!(beta > 0) || !(eta > 0 && eta < 1)) return fail(TG_EINVAL, "need beta > 0 and 0 < eta < 1");
  hipStream_t s = (hipStream_t)stream;
  k_filter<<<nblocks(n_elem(g)), TO_BLOCK, 0, s>>>(x_d, g->nx, g->ny, g->nz, stencil_R(r_min), r_min, beta, eta,
                                                     xt_d, xbar_d, dxbar_d);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int tg_oc_update(const tg_grid* g, const double* x_d, const double* dc_d, const double* dv_d, double volfrac,
                 double move, double r_min, double beta, double eta, double* x_new_d, double* lambda_h,
                 void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_r(r_min))) return rc;
  if (!x_d || !dc_d || !dv_d || !x_new_d) return fail(TG_EINVAL, "NULL argument");
  if (!(volfrac > 0 && volfrac < 1) || !(move > 0) || !(beta > 0) || !(eta > 0 && eta < 1))
    return fail(TG_EINVAL, "need 0 < volfrac < 1, move > 0, beta > 0, 0 < eta < 1");
  return oc_update(g, x_d, dc_d, dv_d, volfrac, move, r_min, beta, eta, x_new_d, lambda_h, (hipStream_t)stream);
}

void tg_default_topopt(tg_topopt_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_iters = 40;
  o->min_iters = 20;
  o->tol = 0.01;
  o->volfrac = 0.30;
  o->r_min = 1.5;
  o->eta = 0.5;
  o->n_stages = 2;
  o->stages[0] = {1, 1.5, 1.0, 0.20};
  o->stages[1] = {16, 3.5, 4.0, 0.15};
  o->mode = TG_LOOP_GUARDED;
  o->fixed_floor = 1e-3;
  tg_default_policy(&o->policy);
  o->policy.n_rungs = 3;
  o->policy.rungs[0] = 1e-12;
  o->policy.rungs[1] = 1e-3;
  o->policy.rungs[2] = 1e-2;
}

int tg_topopt_workspace_bytes(const tg_grid* g, size_t* bytes) {
  if (!g || !bytes) return fail(TG_EINVAL, "NULL argument");
  const size_t ne = (size_t)g->nx * g->ny * g->nz, nd = (size_t)g->lv[0].n_dof;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  *bytes = 7 * al(ne * sizeof(double)) + al(nd * sizeof(double));
  return TG_OK;
}

int tg_topopt_run(tg_grid* g, const double* f_d, const tg_topopt_opts* o, void* ws_d, size_t ws_bytes,
                  double* x_d, tg_topopt_record* rec, int* n_rec, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!f_d || !o || !ws_d || !x_d || !rec || !n_rec) return fail(TG_EINVAL, "NULL argument");
  if ((rc = check_r(o->r_min))) return rc;
  if (o->n_stages < 1 || o->n_stages > 4 || o->stages[0].first_iter != 1 || o->max_iters < 1)
    return fail(TG_EINVAL, "need 1..4 continuation stages, the first starting at iteration 1");
  if (o->mode < TG_LOOP_GUARDED || o->mode > TG_LOOP_FIXED) return fail(TG_EINVAL, "bad loop mode");
  size_t need = 0;
  tg_topopt_workspace_bytes(g, &need);
  if (ws_bytes < need) return fail(TG_EWORKSPACE, "topopt workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const size_t ne = (size_t)n_elem(g);
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* w = (char*)ws_d;
  double* B[7];
  for (int i = 0; i < 7; ++i, w += al(ne * sizeof(double))) B[i] = (double*)w;
  double *xt = B[0], *xbar = B[1], *dxbar = B[2], *dcp = B[3], *dcd = B[4], *dv = B[5], *xn = B[6];
  double* u = (double*)w;
  const double r = o->r_min, eta = o->eta;
  const tg_policy& pol0 = o->policy;
  int prev_rung = -1;
  *n_rec = 0;
  for (int t = 1; t <= o->max_iters; ++t) {
    const auto t0 = std::chrono::steady_clock::now();
    int st = 0;
    for (int q = 0; q < o->n_stages; ++q)
      if (t >= o->stages[q].first_iter) st = q;
    const double p = o->stages[st].p, beta = o->stages[st].beta, move = o->stages[st].move;
    tg_topopt_record& R = rec[t - 1];
    std::memset(&R, 0, sizeof(R));
    R.iter = t;
    R.p = p;
    R.beta = beta;
    if ((rc = tg_filter_project(g, x_d, r, beta, eta, xt, xbar, dxbar, stream))) return rc;
    // the state solve
    tg_policy pol = pol0;
    pol.p = p;
    double floor = -1.0;
    if (o->mode == TG_LOOP_FIXED) {
      if ((rc = tg_set_density(g, xbar, p, o->fixed_floor, stream))) return rc;
      tg_solve_result sr;
      if ((rc = tg_fgmres_solve(g, f_d, u, &pol.solve, &sr, nullptr, stream))) return rc;
      if ((rc = tg_true_residual(g, f_d, u, &R.true_eta, stream))) return rc;
      R.solve_iters = sr.iterations;
      R.accepted = -1;           // no acceptance test
      R.rung = -1;
      floor = o->fixed_floor;
    } else {
      bool done = false;
      if (o->mode == TG_LOOP_REUSE && prev_rung >= 0) {
        // the previous decision, kept while the guard accepts it
        if ((rc = tg_set_density(g, xbar, p, pol.rungs[prev_rung], stream))) return rc;
        tg_solve_result sr;
        if ((rc = tg_fgmres_solve(g, f_d, u, &pol.solve, &sr, nullptr, stream))) return rc;
        double eta_t = 1.0;
        if ((rc = tg_true_residual(g, f_d, u, &eta_t, stream))) return rc;
        R.solve_iters += sr.iterations;
        if (eta_t <= pol.tau) {
          done = true;
          R.rung = prev_rung;
          R.true_eta = eta_t;
          R.accepted = 1;
          floor = pol.rungs[prev_rung];
        }
      }
      if (!done) {
        tg_policy_result pr;
        if ((rc = tg_select_floor(g, xbar, f_d, &pol, u, &pr, stream))) return rc;
        R.probed = 1;
        R.solve_iters += pr.iters_probe + pr.iters_selected + pr.iters_rejected;
        R.rung = pr.rung;
        if (pr.rung < 0) {
          R.accepted = 0;
          *n_rec = t;
          return TG_OK;          // no admissible floor: the loop stops here
        }
        R.true_eta = pr.attempts[pr.n_attempts - 1].true_eta;
        R.accepted = 1;
        floor = pr.floor;
        prev_rung = pr.rung;
      }
    }
    R.floor = floor;
    // compliance and its gradient with respect to the design
    if ((rc = tg_compliance_sensitivity(g, xbar, p, floor, f_d, u, nullptr, dcp, &R.compliance, stream))) return rc;
    if ((rc = tg_density_filter_adjoint(g, dcp, dxbar, r, dcd, stream))) return rc;
    if ((rc = tg_density_filter_adjoint(g, dxbar, nullptr, r, dv, stream))) return rc;
    if ((rc = oc_update(g, x_d, dcd, dv, o->volfrac, move, r, beta, eta, xn, nullptr, s))) return rc;
    double vol = 0.0;
    // volume of the physical density this iteration solved with, and the
    // largest design change of the step
    if ((rc = reduce_host(g, x_d, nullptr, r, beta, eta, 0, s, &vol))) return rc;
    R.volume = vol / (double)ne;
    if ((rc = reduce_host(g, xn, x_d, r, beta, eta, 1, s, &R.change))) return rc;
    TG_HIP(hipMemcpyAsync(x_d, xn, ne * sizeof(double), hipMemcpyDeviceToDevice, s));
    TG_HIP(hipStreamSynchronize(s));
    R.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *n_rec = t;
    if (t >= o->min_iters && R.change < o->tol) break;
  }
  return TG_OK;
}

}  // extern "C"
