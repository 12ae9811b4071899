// Compliance, compliance sensitivities and the comparison of two gradient
// fields: what a raised floor changes in the quantities an optimizer reads
// (sensitivity expression of Sec. 3.1; Sec. 4.4.1, Tab. perturbation).
//
// k_energy_sens marches element columns in z like the operator kernels: a
// workgroup owns 16 x 16 columns and a run of element layers, each thread
// keeps the bottom face of its element in registers and loads only the new
// top face per layer (coalesced along x, neighbouring columns share lines in
// L1/L2).  Each face is taken into the per-component Walsh basis once; in
// that basis the cube's element stiffness has eight distinct coefficients,
// so u_e^T K_e u_e is a 30-term quadratic form instead of a 24 x 24
// contraction.  The compliance f^T u rides along: every node is counted by
// exactly one thread.  All sums use fixed orders, so results are bitwise
// reproducible.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tg_internal.h"

namespace tg {
namespace {

constexpr int EN_T = 16;        // element columns per tile edge
constexpr int GM_BLOCKS = 1024; // workgroups of the gradient-moment sweeps
constexpr int GM_VALS = 6;      // partial sums per workgroup

// Entries of H K_e H^T / 64 (H[m][a] = product over the bits b of m of +1 for
// a_b = 1, -1 for a_b = 0; index 3 m + component): d, o on the three normal
// modes (x-mode of u_x, y-mode of u_y, z-mode of u_z), s on the three shear
// pairs, p, q on the three bilinear pairs, r, t on the three bilinear modes
// of the remaining component, w on the trilinear mode; zero elsewhere.
struct EnCoef {
  double d, o, s, p, q, r, t, w;
};

// x and y stages of the transform on one z-face, corner c = di + 2 dj.
__device__ __forceinline__ void face_walsh(double* v) {
  const double a0 = v[0] + v[1], a1 = v[1] - v[0], a2 = v[2] + v[3], a3 = v[3] - v[2];
  v[0] = a0 + a2;
  v[1] = a1 + a3;
  v[2] = a2 - a0;
  v[3] = a3 - a1;
}

// u_e^T K_e u_e from the element's modes X, Y, Z (mode m = mx + 2 my + 4 mz).
__device__ __forceinline__ double energy_form(const double* X, const double* Y, const double* Z,
                                              const EnCoef& c) {
  const double n0 = X[1], n1 = Y[2], n2 = Z[4];
  double e = c.d * (n0 * n0 + n1 * n1 + n2 * n2) + 2.0 * c.o * (n0 * n1 + n0 * n2 + n1 * n2);
  const double s0 = Y[1] + X[2], s1 = Z[1] + X[4], s2 = Z[2] + Y[4];
  e += c.s * (s0 * s0 + s1 * s1 + s2 * s2);
  const double pa[3] = {X[3], Y[3], X[5]}, pb[3] = {Z[6], Z[5], Y[6]};
#pragma unroll
  for (int i = 0; i < 3; ++i) e += c.p * (pa[i] * pa[i] + pb[i] * pb[i]) + 2.0 * c.q * (pa[i] * pb[i]);
  const double t0 = Z[3], t1 = Y[5], t2 = X[6];
  e += c.r * (t0 * t0 + t1 * t1 + t2 * t2) + 2.0 * c.t * (t0 * t1 + t0 * t2 + t1 * t2);
  e += c.w * (X[7] * X[7] + Y[7] * Y[7] + Z[7] * Z[7]);
  return e;
}

// Fixed-order sum over the 256 threads of a workgroup; thread 0 gets it.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

// energy[e] = u_e^T K_e u_e, dc[e] = coef rho_e^pm1 energy (coef = -p (1 -
// rho_min), pm1 = p - 1) for the element layers [z0, z0 + zc) of this tile;
// part[block] = this block's share of f^T u (f may be NULL).  Clamped nodes
// (i = 0) read as zero.  Grid: (tiles, z chunks), 256 threads.
__global__ __launch_bounds__(256) void k_energy_sens(const double* __restrict__ u,
                                                     const double* __restrict__ f,
                                                     const double* __restrict__ rho, int nx, int ny,
                                                     int nz, int zc, double coef, double pm1, EnCoef c,
                                                     double* __restrict__ energy,
                                                     double* __restrict__ dc,
                                                     double* __restrict__ part) {
  __shared__ double red[4];
  const int tx = threadIdx.x & (EN_T - 1), ty = threadIdx.x / EN_T;
  const int ntx = (nx + EN_T - 1) / EN_T;
  const int ex = (int)(blockIdx.x % ntx) * EN_T + tx, ey = (int)(blockIdx.x / ntx) * EN_T + ty;
  const int z0 = (int)blockIdx.y * zc, z1 = min(nz, z0 + zc);
  const long long NX = nx + 1, NXY = (long long)(nx + 1) * (ny + 1);
  double fu = 0.0;
  if (ex < nx && ey < ny) {
    // corner (di, dj) of the faces is this thread's node for the compliance
    // when no other column holds it as its corner (0, 0)
    bool own[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) own[q] = ((q & 1) == 0 || ex == nx - 1) && ((q >> 1) == 0 || ey == ny - 1);
    auto load_face = [&](int k, double* X, double* Y, double* Z, bool count) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ex + (q & 1);
        const long long n = i + NX * (ey + (q >> 1)) + NXY * k;
        if (i == 0) {
          X[q] = Y[q] = Z[q] = 0.0;
        } else {
          X[q] = u[3 * n];
          Y[q] = u[3 * n + 1];
          Z[q] = u[3 * n + 2];
          if (f && count && own[q]) fu += f[3 * n] * X[q] + f[3 * n + 1] * Y[q] + f[3 * n + 2] * Z[q];
        }
      }
      face_walsh(X);
      face_walsh(Y);
      face_walsh(Z);
    };
    double bx[4], by[4], bz[4];
    load_face(z0, bx, by, bz, z0 == 0);
    for (int k = z0; k < z1; ++k) {
      double tx4[4], ty4[4], tz4[4];
      load_face(k + 1, tx4, ty4, tz4, true);
      double X[8], Y[8], Z[8];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        X[m] = tx4[m] + bx[m];
        X[m + 4] = tx4[m] - bx[m];
        Y[m] = ty4[m] + by[m];
        Y[m + 4] = ty4[m] - by[m];
        Z[m] = tz4[m] + bz[m];
        Z[m + 4] = tz4[m] - bz[m];
      }
      const double en = energy_form(X, Y, Z, c);
      const long long e = ex + (long long)nx * (ey + (long long)ny * k);
      if (energy) energy[e] = en;
      if (dc) dc[e] = coef * pow(rho[e], pm1) * en;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        bx[m] = tx4[m];
        by[m] = ty4[m];
        bz[m] = tz4[m];
      }
    }
  }
  const double s = block_sum(fu, red);
  if (part && threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// Moments of two gradient fields over the elements with rho >= solid_min,
// GM_VALS partials per workgroup (fixed element-to-thread assignment).
// pass 0: count, sum g0, sum g1.  pass 1 (means m0, m1 given): centred
// sum (g0 - m0)^2, sum (g1 - m1)^2, sum (g0 - m0)(g1 - m1), sum (g1 - g0)^2,
// and the plain sums g0^2, g1^2.
__global__ __launch_bounds__(256) void k_grad_moments(const double* __restrict__ rho, double solid_min,
                                                      const double* __restrict__ g0,
                                                      const double* __restrict__ g1, long long n,
                                                      int pass, double m0, double m1,
                                                      double* __restrict__ part) {
  __shared__ double red[4];
  double a[GM_VALS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    if (!(rho[e] >= solid_min)) continue;
    const double x = g0[e], y = g1[e];
    if (pass == 0) {
      a[0] += 1.0;
      a[1] += x;
      a[2] += y;
    } else {
      const double dx = x - m0, dy = y - m1, df = y - x;
      a[0] += dx * dx;
      a[1] += dy * dy;
      a[2] += dx * dy;
      a[3] += df * df;
      a[4] += x * x;
      a[5] += y * y;
    }
  }
#pragma unroll
  for (int q = 0; q < GM_VALS; ++q) {
    const double s = block_sum(a[q], red);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * GM_VALS + q] = s;
  }
}

}  // namespace
}  // namespace tg

using namespace tg;

extern "C" {

int tg_compliance_sensitivity(const tg_grid* g, const double* rho_d, double p, double rho_min,
                              const double* f_d, const double* u_d, double* energy_d, double* dc_d,
                              double* compliance_h, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!u_d) return fail(TG_EINVAL, "u_d is NULL");
  if (!energy_d && !dc_d && !compliance_h) return fail(TG_EINVAL, "no output requested");
  if (dc_d && !rho_d) return fail(TG_EINVAL, "sensitivities need rho_d");
  if (compliance_h && !f_d) return fail(TG_EINVAL, "compliance needs f_d");
  if (!(p > 0) || !std::isfinite(p) || !(rho_min >= 0 && rho_min <= 1))
    return fail(TG_EINVAL, "need p > 0 and 0 <= rho_min <= 1");
  hipStream_t s = (hipStream_t)stream;
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const int tiles = ((nx + EN_T - 1) / EN_T) * ((ny + EN_T - 1) / EN_T);
  // enough z chunks for about 2048 workgroups; each chunk re-reads one face
  const int want = std::max(1, std::min(nz, (2048 + tiles - 1) / tiles));
  const int zc = (nz + want - 1) / want, nzc = (nz + zc - 1) / zc;
  const long long nblk = (long long)tiles * nzc;
  if (nblk > (long long)TG_PART_W * g->lv[0].n_chunks || nzc > 65535)
    return fail(TG_EINVAL, "grid too large for the partial-sum buffer");
  const ModeCoef<double>& m = g->mc64;
  const EnCoef c = {m.d, m.o, m.s, m.p, m.q, m.r, m.t, m.w};
  double* part = g->desc.part;
  const double nodes = (double)g->lv[0].n_nodes, elems = (double)nx * ny * nz;
  const double bytes = 24.0 * nodes * (1.0 + (compliance_h ? 1.0 : 0.0)) +
                       elems * ((dc_d ? 16.0 : 0.0) + (energy_d ? 8.0 : 0.0));
  void* th = timer_begin(TG_KT_FIDELITY, s);
  k_energy_sens<<<dim3((unsigned)tiles, (unsigned)nzc), 256, 0, s>>>(
      u_d, compliance_h ? f_d : nullptr, rho_d, nx, ny, nz, zc, -p * (1.0 - rho_min), p - 1.0, c,
      energy_d, dc_d, part);
  if (th) timer_end(th, bytes, s);
  TG_HIP(hipGetLastError());
  if (compliance_h) {
    std::vector<double> h((size_t)nblk);
    TG_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * nblk, hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
    double sum = 0.0;
    for (double v : h) sum += v;
    *compliance_h = sum;
  }
  return TG_OK;
}

int tg_gradient_change(const tg_grid* g, const double* rho_d, double solid_min, const double* dc0_d,
                       const double* dc1_d, tg_gradient_change_result* out, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!rho_d || !dc0_d || !dc1_d || !out) return fail(TG_EINVAL, "NULL argument");
  if (!std::isfinite(solid_min)) return fail(TG_EINVAL, "solid_min must be finite");
  hipStream_t s = (hipStream_t)stream;
  const long long n = (long long)g->nx * g->ny * g->nz;
  const int nblk = (int)std::min<long long>(GM_BLOCKS, (n + 255) / 256);
  if ((long long)nblk * GM_VALS > (long long)TG_PART_W * g->lv[0].n_chunks)
    return fail(TG_EINVAL, "grid too small for the partial-sum buffer");
  double* part = g->desc.part;
  std::vector<double> h((size_t)nblk * GM_VALS);
  double acc[GM_VALS];
  auto sweep = [&](int pass, double m0, double m1) -> int {
    void* th = timer_begin(TG_KT_FIDELITY, s);
    k_grad_moments<<<nblk, 256, 0, s>>>(rho_d, solid_min, dc0_d, dc1_d, n, pass, m0, m1, part);
    if (th) timer_end(th, 24.0 * (double)n, s);
    TG_HIP(hipGetLastError());
    TG_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < GM_VALS; ++q) {
      acc[q] = 0.0;
      for (int b = 0; b < nblk; ++b) acc[q] += h[(size_t)b * GM_VALS + q];
    }
    return TG_OK;
  };
  int rc = sweep(0, 0.0, 0.0);
  if (rc) return rc;
  const double cnt = acc[0];
  if (cnt < 1) return fail(TG_EINVAL, "no element has rho >= solid_min");
  rc = sweep(1, acc[1] / cnt, acc[2] / cnt);
  if (rc) return rc;
  out->n_solid = (int64_t)cnt;
  out->norm0 = std::sqrt(acc[4]);
  out->norm1 = std::sqrt(acc[5]);
  out->rel_l2 = std::sqrt(acc[3]) / out->norm0;
  out->pearson = acc[2] / std::sqrt(acc[0] * acc[1]);
  return TG_OK;
}

}  // extern "C"
