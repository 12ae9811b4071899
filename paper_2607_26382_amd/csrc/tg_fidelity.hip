// Compliance, compliance sensitivities and the comparison of two gradient
// fields: what a raised floor changes in the quantities an optimizer reads
// (sensitivity expression of Sec. 3.1; Sec. 4.4.1, Tab. perturbation).
//
// k_energy_sens marches element columns in z like the operator kernels: a
// workgroup owns 16 x 16 columns and a run of element layers; each node
// layer is loaded once (coalesced, one layer ahead) and staged in LDS, and
// each thread keeps the bottom face of its element from the previous layer.
// Faces are taken into the per-component Walsh basis once; in that basis the
// cube's element stiffness has eight distinct coefficients, so u_e^T K_e u_e
// is a 30-term quadratic form instead of a 24 x 24 contraction.  The
// compliance f^T u rides along at staging, every node counted by exactly one
// workgroup.  All sums use fixed orders, so results are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <mutex>
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

// dc[e] = rho_e^pm1 for exponents that are not whole or half-whole (the
// energy pass then scales it in place).
__global__ __launch_bounds__(256) void k_rho_pow(const double* __restrict__ rho, double pm1, long long n,
                                                 double* __restrict__ dc) {
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256)
    dc[e] = pow(rho[e], pm1);
}

// energy[e] = u_e^T K_e u_e, dc[e] = coef rho_e^(p - 1) energy (coef = -p (1 -
// rho_min)) for the element layers [z0, z0 + zc) of this tile; the power is
// rho^ipm1 (times sqrt(rho) if half) as a product when ipm1 >= 0, else dc
// already holds it (k_rho_pow); part[block] = this block's share of f^T u
// (f may be NULL).
// Clamped nodes (i = 0) read as zero.  Grid: (tiles, z chunks), 256 threads.
//
// Each node layer of the tile (17 x 17 nodes, rows contiguous in memory) is
// loaded once, coalesced, two nodes per thread, one layer ahead of its use,
// and staged in LDS; a thread reads its element's four top corners there and
// keeps the bottom face, already in modes, from the previous layer.  The
// staging thread of a node also adds its f.u when the tile owns the node
// (x, y in the tile's half-open range, or the grid's last plane), once per
// node layer.
__global__ __launch_bounds__(256) void k_energy_sens(const double* __restrict__ u,
                                                     const double* __restrict__ f,
                                                     const double* __restrict__ rho, int nx, int ny,
                                                     int nz, int zc, double coef, int ipm1, int half,
                                                     EnCoef c, double* __restrict__ energy,
                                                     double* __restrict__ dc,
                                                     double* __restrict__ part) {
  constexpr int NT = EN_T + 1;            // nodes per tile edge
  __shared__ double su[2][3][NT][NT];   // node layers, alternating
  __shared__ double red[4];
  const int tx = threadIdx.x & (EN_T - 1), ty = threadIdx.x / EN_T;
  const int ntx = (nx + EN_T - 1) / EN_T;
  // logical block (tile, z chunk) = tile + tiles * chunk, dealt so that each
  // XCD runs a contiguous range: neighbouring tiles share their halo nodes
  // and partly used cache lines in one L2
  const int nb = (int)(gridDim.x * gridDim.y);
  const int lb = xcd_tile((int)(blockIdx.x + gridDim.x * blockIdx.y), nb);
  const int tile = lb % (int)gridDim.x, chunk = lb / (int)gridDim.x;
  const int x0 = (tile % ntx) * EN_T, y0 = (tile / ntx) * EN_T;
  const int ex = x0 + tx, ey = y0 + ty;
  const int z0 = chunk * zc, z1 = min(nz, z0 + zc);
  const long long NX = nx + 1, NXY = (long long)(nx + 1) * (ny + 1);
  const bool act = ex < nx && ey < ny;
  // the two staged nodes of this thread: q = threadIdx.x + 256 s, (lx, ly)
  int gn[2];                      // node index within a layer, -1 if none
  bool ownq[2];
#pragma unroll
  for (int sI = 0; sI < 2; ++sI) {
    const int q = threadIdx.x + 256 * sI, lx = q % NT, ly = q / NT;
    const int i = x0 + lx, j = y0 + ly;
    const bool in = q < NT * NT && i <= nx && j <= ny;
    gn[sI] = (in && i > 0) ? (int)(i + NX * j) : -1;   // clamped nodes stay zero
    ownq[sI] = in && (lx < EN_T || i == nx) && (ly < EN_T || j == ny);
  }
  double fu = 0.0;
  double pv[2][3], pf[2][3];
  auto fetch = [&](int k) {
#pragma unroll
    for (int sI = 0; sI < 2; ++sI) {
      const long long n = gn[sI] >= 0 ? gn[sI] + NXY * k : -1;
#pragma unroll
      for (int cI = 0; cI < 3; ++cI) {
        pv[sI][cI] = n >= 0 ? u[3 * n + cI] : 0.0;
        pf[sI][cI] = (f && n >= 0 && ownq[sI]) ? f[3 * n + cI] : 0.0;
      }
    }
  };
  auto stage = [&](int buf, bool count) {
#pragma unroll
    for (int sI = 0; sI < 2; ++sI) {
      const int q = threadIdx.x + 256 * sI;
      if (q < NT * NT) {
#pragma unroll
        for (int cI = 0; cI < 3; ++cI) su[buf][cI][q / NT][q % NT] = pv[sI][cI];
        if (count) fu += pf[sI][0] * pv[sI][0] + pf[sI][1] * pv[sI][1] + pf[sI][2] * pv[sI][2];
      }
    }
  };
  auto read_face = [&](int buf, double* X, double* Y, double* Z) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      X[q] = su[buf][0][ty + (q >> 1)][tx + (q & 1)];
      Y[q] = su[buf][1][ty + (q >> 1)][tx + (q & 1)];
      Z[q] = su[buf][2][ty + (q >> 1)][tx + (q & 1)];
    }
    face_walsh(X);
    face_walsh(Y);
    face_walsh(Z);
  };
  double bx[4], by[4], bz[4];
  // node layer k lives in su[(k - z0) & 1]: the layer staged in step k goes
  // to the buffer last read two steps earlier, so the barrier of the step
  // between separates them and one barrier per layer suffices
  fetch(z0);
  stage(0, z0 == 0);
  fetch(z0 + 1);
  __syncthreads();
  read_face(0, bx, by, bz);
  for (int k = z0; k < z1; ++k) {
    const long long ek = ex + (long long)nx * (ey + (long long)ny * k);
    const double rk = (act && dc) ? (ipm1 >= 0 ? rho[ek] : dc[ek]) : 0.0;
    const int nb1 = (k + 1 - z0) & 1;
    stage(nb1, true);           // node layer k + 1
    if (k + 1 < z1) fetch(k + 2);
    __syncthreads();
    double tx4[4], ty4[4], tz4[4];
    read_face(nb1, tx4, ty4, tz4);
    if (act) {
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
      if (dc) {
        double rp = rk;
        if (ipm1 >= 0) {
          rp = 1.0;
          for (int t = 0; t < ipm1; ++t) rp *= rk;
          if (half) rp *= sqrt(rk);
        }
        dc[e] = coef * rp * en;
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      bx[m] = tx4[m];
      by[m] = ty4[m];
      bz[m] = tz4[m];
    }
  }
  const double sum = block_sum(fu, red);
  if (part && threadIdx.x == 0) part[lb] = sum;   // summed on the host in logical order
}

// Moments of two gradient fields over the elements with rho >= solid_min,
// GM_VALS partials per workgroup (fixed element-to-thread assignment).
// pass 0: count, sum g0, sum g1.  pass 1 (means m0, m1 given): centred
// sum (g0 - m0)^2, sum (g1 - m1)^2, sum (g0 - m0)(g1 - m1), sum (g1 - g0)^2,
// and the plain sums g0^2, g1^2.
// mean_d (may be null): the two means read from device memory instead of
// m0, m1 (the allocation-free path keeps them on the device between passes).
__global__ __launch_bounds__(256) void k_grad_moments(const double* __restrict__ rho, double solid_min,
                                                      const double* __restrict__ g0,
                                                      const double* __restrict__ g1, long long n,
                                                      int pass, double m0, double m1,
                                                      const double* __restrict__ mean_d,
                                                      double* __restrict__ part) {
  __shared__ double red[4];
  if (mean_d) {
    m0 = mean_d[0];
    m1 = mean_d[1];
  }
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

// One lane sums the nblk x GM_VALS partials of a moment pass in block order
// (the order the host-side sum of tg_gradient_change uses) into
// tot[GM_VALS * pass + q]; after pass 0 the two means follow in
// tot[2 * GM_VALS], tot[2 * GM_VALS + 1] (0 when no element is solid).
__global__ void k_grad_finish(const double* __restrict__ part, int nblk, int pass, double* __restrict__ tot) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc[GM_VALS];
  for (int q = 0; q < GM_VALS; ++q) {
    acc[q] = 0.0;
    for (int b = 0; b < nblk; ++b) acc[q] += part[(long long)b * GM_VALS + q];
    tot[GM_VALS * pass + q] = acc[q];
  }
  if (pass == 0) {
    const double cnt = acc[0];
    tot[2 * GM_VALS] = cnt >= 1 ? acc[1] / cnt : 0.0;
    tot[2 * GM_VALS + 1] = cnt >= 1 ? acc[2] / cnt : 0.0;
  }
}

// Reduction scratch of the allocation-free comparison: the per-workgroup
// partials of one pass, then the totals of both passes and the two means.
// One copy per GPU, held until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
constexpr int NA_PART = GM_BLOCKS * GM_VALS;
constexpr int NA_DOUBLES = NA_PART + 2 * GM_VALS + 2;
static_assert(NA_DOUBLES * sizeof(double) == TG_NOALLOC_SCRATCH_BYTES, "scratch size in the header");
__device__ __align__(256) double scratch[NA_DOUBLES];

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mu;
double* na_ptr[NA_MAX_DEVICES] = {};

// The device address of `scratch` on the current device (looked up once per
// device, with that device current).
int noalloc_scratch(double** out) {
  int dev = -1;
  TG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NA_MAX_DEVICES) return fail(TG_EINVAL, "device index beyond the library's table");
  std::lock_guard<std::mutex> lk(na_mu);
  if (!na_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    na_ptr[dev] = static_cast<double*>(p);
  }
  *out = na_ptr[dev];
  return TG_OK;
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
  // enough z chunks for about 1024 workgroups; each chunk re-reads one face
  const int want = std::max(1, std::min(nz, (1024 + tiles - 1) / tiles));
  const int zc = (nz + want - 1) / want, nzc = (nz + zc - 1) / zc;
  const long long nblk = (long long)tiles * nzc;
  if (nblk > (long long)TG_PART_W * g->lv[0].n_chunks || nzc > 65535)
    return fail(TG_EINVAL, "grid too large for the partial-sum buffer");
  // whole and half-whole exponents p - 1 <= 8 as products (times a square
  // root), others by a separate power pass into dc
  const double pm1 = p - 1.0;
  const bool prod = pm1 >= 0 && pm1 <= 8 && 2 * pm1 == std::floor(2 * pm1);
  const int ipm1 = prod ? (int)std::floor(pm1) : -1, half = prod && pm1 != std::floor(pm1);
  const ModeCoef<double>& m = g->mc64;
  const EnCoef c = {m.d, m.o, m.s, m.p, m.q, m.r, m.t, m.w};
  double* part = g->desc.part;
  const double nodes = (double)g->lv[0].n_nodes, elems = (double)nx * ny * nz;
  const double bytes = 24.0 * nodes * (1.0 + (compliance_h ? 1.0 : 0.0)) +
                       elems * ((dc_d ? 16.0 : 0.0) + (energy_d ? 8.0 : 0.0));
  if (dc_d && !prod) {
    const long long ne = (long long)nx * ny * nz;
    void* tp = timer_begin(TG_KT_FIDELITY, s);
    k_rho_pow<<<(int)std::min<long long>(4096, (ne + 255) / 256), 256, 0, s>>>(rho_d, pm1, ne, dc_d);
    if (tp) timer_end(tp, 16.0 * (double)ne, s);
    TG_HIP(hipGetLastError());
  }
  void* th = timer_begin(TG_KT_FIDELITY, s);
  k_energy_sens<<<dim3((unsigned)tiles, (unsigned)nzc), 256, 0, s>>>(
      u_d, compliance_h ? f_d : nullptr, dc_d ? rho_d : nullptr, nx, ny, nz, zc, -p * (1.0 - rho_min), ipm1,
      half, c, energy_d, dc_d, part);
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
    k_grad_moments<<<nblk, 256, 0, s>>>(rho_d, solid_min, dc0_d, dc1_d, n, pass, m0, m1, nullptr, part);
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

int tg_gradient_change_noalloc(int64_t n_elem, const double* rho_d, double solid_min, const double* dc0_d,
                               const double* dc1_d, tg_gradient_change_result* out, void* stream) {
  if (!rho_d || !dc0_d || !dc1_d || !out) return fail(TG_EINVAL, "NULL argument");
  if (n_elem < 1 || n_elem > TG_NOALLOC_MAX_ELEMS)
    return fail(TG_EINVAL, "n_elem must be in [1, TG_NOALLOC_MAX_ELEMS]");
  if (!std::isfinite(solid_min)) return fail(TG_EINVAL, "solid_min must be finite");
  double* sc = nullptr;
  int rc = noalloc_scratch(&sc);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const long long n = (long long)n_elem;
  const int nblk = (int)std::min<long long>(GM_BLOCKS, (n + 255) / 256);
  double* part = sc;
  double* tot = sc + NA_PART;
  // every partial and total read below is written earlier in the same call
  // (k_grad_moments writes all nblk x GM_VALS partials it is launched with)
  for (int pass = 0; pass < 2; ++pass) {
    void* th = timer_begin(TG_KT_FIDELITY, s);
    k_grad_moments<<<nblk, 256, 0, s>>>(rho_d, solid_min, dc0_d, dc1_d, n, pass, 0.0, 0.0,
                                        pass ? tot + 2 * GM_VALS : nullptr, part);
    if (th) timer_end(th, 24.0 * (double)n, s);
    TG_HIP(hipGetLastError());
    k_grad_finish<<<1, 64, 0, s>>>(part, nblk, pass, tot);
    TG_HIP(hipGetLastError());
  }
  double acc[2 * GM_VALS];
  TG_HIP(hipMemcpyAsync(acc, tot, sizeof(acc), hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  const double cnt = acc[0];
  if (cnt < 1) return fail(TG_EINVAL, "no element has rho >= solid_min");
  const double* c = acc + GM_VALS;
  out->n_solid = (int64_t)cnt;
  out->norm0 = std::sqrt(c[4]);
  out->norm1 = std::sqrt(c[5]);
  out->rel_l2 = std::sqrt(c[3]) / out->norm0;
  out->pearson = c[2] / std::sqrt(c[0] * c[1]);
  return TG_OK;
}

}  // extern "C"
