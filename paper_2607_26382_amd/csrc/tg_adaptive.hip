// The fine-level adaptive correction of the paper's preconditioner (Tab.
// solver-config) and the flexible GMRES around it (Sec. 3.5).
//
// One application z = M(v): z = V-cycle(v); with s = v - K z, an inner
// right-preconditioned GMRES (restart = steps = q, stopping only on breakdown
// or a non-finite value) solves K d = s from d = 0 with the 3 x 3 node-block
// Jacobi operator as its preconditioner; z + d replaces z only if
// ||s - K d|| < ||s||.  M depends on v nonlinearly (the accept test, the inner
// Krylov polynomial), so the outer method stores the preconditioned vectors
// Z and forms x = x0 + Z y (flexible GMRES, Saad 1993).
//
// The path is single-grid.  The outer iteration reads each Hessenberg column
// back to the host; the inner iteration of the correction keeps its scalar
// work (rotations, least squares, accept test) on the device, so one
// application of M needs no host synchronization.  K is the library's FP64
// operator, the V-cycle runs at the
// requested precision (FP32 forms through float copies), the node-block
// inverses are the smoother's.  Sums run in a fixed order (block partials,
// then one wavefront per sum), so results are reproducible run to run.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <vector>

#include "tg_internal.h"

namespace tg {
namespace {

constexpr int AD_BLOCK = 256;
constexpr int AD_QG = 8;            // basis vectors per workgroup of the multi-dot
constexpr int AD_MAXB = 1024;       // workgroups of the vector kernels
constexpr int AD_MAXV = TG_AD_MAX_RESTART + 1;

int nblk(long long n) { return (int)std::max<long long>(1, std::min<long long>(AD_MAXB, (n + AD_BLOCK - 1) / AD_BLOCK)); }
// multi-dot workgroups: at least four elements per thread, so the partials
// stay few (one wavefront sums them)
int nblk_dots(long long n) {
  return (int)std::max<long long>(1, std::min<long long>(AD_MAXB, (n + 4 * AD_BLOCK - 1) / (4 * AD_BLOCK)));
}
size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
long long ld_of(long long n) { return (n + 31) & ~31LL; }   // doubles per basis vector (256-byte rows)

// part[q * gridDim.x + block] = sum over the block's strided range of V_q[i] w[i]
// for q < nv, and (with_self) of w[i]^2 for q = nv
__global__ __launch_bounds__(AD_BLOCK) void k_ad_dots(const double* __restrict__ V, long long ld, int nv,
                                                      int with_self, const double* __restrict__ w, long long n,
                                                      double* __restrict__ part) {
  const int nt = nv + with_self;
  __shared__ double red[AD_BLOCK / 64][AD_QG];
  const int q0 = blockIdx.y * AD_QG;
  double acc[AD_QG];
#pragma unroll
  for (int t = 0; t < AD_QG; ++t) acc[t] = 0.0;
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK) {
    const double wi = w[i];
#pragma unroll
    for (int t = 0; t < AD_QG; ++t) {
      if (q0 + t < nv) acc[t] += V[(long long)(q0 + t) * ld + i] * wi;
      else if (q0 + t == nv && with_self) acc[t] += wi * wi;
    }
  }
#pragma unroll
  for (int t = 0; t < AD_QG; ++t) {
    double s = acc[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][t] = s;
  }
  __syncthreads();
  if (threadIdx.x < AD_QG && q0 + (int)threadIdx.x < nt) {
    double s = 0.0;
    for (int w8 = 0; w8 < AD_BLOCK / 64; ++w8) s += red[w8][threadIdx.x];
    part[(long long)(q0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
  }
}

// out[q] = sum_b part[q nb + b], one wavefront per q (lane-strided partial
// sums, then a butterfly; a fixed order for a given block count); h[q] =
// out[q] (acc = 0) or h[q] + out[q] (acc = 1); the sum q = nv (if the grid
// has it) goes to *self_out
__global__ __launch_bounds__(64) void k_ad_sum(const double* __restrict__ part, int nb, int nv,
                                               double* __restrict__ out, double* __restrict__ h, int acc,
                                               double* __restrict__ self_out) {
  const int q = blockIdx.x;
  double s = 0.0;
#pragma unroll 4
  for (int b = threadIdx.x; b < nb; b += 64) s += part[(long long)q * nb + b];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x == 0) {
    if (q == nv) {
      *self_out = s;
      return;
    }
    out[q] = s;
    if (h) h[q] = acc ? h[q] + s : s;
  }
}

// w += sgn * sum_q c[q] V_q
__global__ __launch_bounds__(AD_BLOCK) void k_ad_update(const double* __restrict__ V, long long ld, int nv,
                                                        const double* __restrict__ c, double sgn,
                                                        double* __restrict__ w, long long n) {
  __shared__ double sc[AD_MAXV];
  for (int q = threadIdx.x; q < nv; q += AD_BLOCK) sc[q] = c[q];
  __syncthreads();
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK) {
    double s = 0.0;
    for (int q = 0; q < nv; ++q) s += sc[q] * V[(long long)q * ld + i];
    w[i] += sgn * s;
  }
}

// w -= sum_q c[q] V_q, and part[block] = the block's sum of the updated
// w[i]^2 (the norm after the last sweep without another pass over w)
__global__ __launch_bounds__(AD_BLOCK) void k_ad_update_norm(const double* __restrict__ V, long long ld, int nv,
                                                             const double* __restrict__ c, double* __restrict__ w,
                                                             long long n, double* __restrict__ part) {
  __shared__ double sc[AD_MAXV];
  __shared__ double red[AD_BLOCK / 64];
  for (int q = threadIdx.x; q < nv; q += AD_BLOCK) sc[q] = c[q];
  __syncthreads();
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK) {
    double s = 0.0;
    for (int q = 0; q < nv; ++q) s += sc[q] * V[(long long)q * ld + i];
    const double wn = w[i] - s;
    w[i] = wn;
    acc += wn * wn;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w8 = 0; w8 < AD_BLOCK / 64; ++w8) s += red[w8];
    part[blockIdx.x] = s;
  }
}

// out = a x + b y (y may be NULL: out = a x); out may alias x or y
__global__ __launch_bounds__(AD_BLOCK) void k_ad_axpby(double a, const double* x, double b, const double* y,
                                                       double* out, long long n) {
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK)
    out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

// z = D^-1 r node by node (D the 3 x 3 diagonal block of K at the node); the
// clamped x = 0 nodes get 0
__global__ __launch_bounds__(AD_BLOCK) void k_ad_jacobi(const double* __restrict__ Dinv, const double* __restrict__ r,
                                                        double* __restrict__ z, long long n_nodes, int NX) {
  for (long long v = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; v < n_nodes;
       v += (long long)gridDim.x * AD_BLOCK) {
    const double r0 = r[3 * v], r1 = r[3 * v + 1], r2 = r[3 * v + 2];
    const double* D = Dinv + 9 * v;
    const bool fixed = (v % NX) == 0;
    z[3 * v] = fixed ? 0.0 : D[0] * r0 + D[1] * r1 + D[2] * r2;
    z[3 * v + 1] = fixed ? 0.0 : D[3] * r0 + D[4] * r1 + D[5] * r2;
    z[3 * v + 2] = fixed ? 0.0 : D[6] * r0 + D[7] * r1 + D[8] * r2;
  }
}

// ---- the inner iteration's scalar work on the device (one lane), so one
// application of the preconditioner needs no host synchronization

// inner state: scalars (IS_*), control ints (stop code, columns done)
enum { IS_R0SQ = 0, IS_INVB = 1, IS_WN0 = 2, IS_HN = 3, IS_INV = 4, IS_R1SQ = 5, IS_ACC = 6, IS_BNORM = 7,
       IS_N = 8 };
enum { IC_STOP = 0, IC_JDONE = 1, IC_N = 4 };

// start of the inner solve on s: beta = ||s|| (from sc[IS_R0SQ]), g = beta e1
__global__ void k_ad_inner_init(double* __restrict__ sc, int* __restrict__ ctl, double* __restrict__ g) {
  const double r0 = sqrt(sc[IS_R0SQ]);
  sc[IS_BNORM] = r0;
  ctl[IC_JDONE] = 0;
  if (r0 == 0.0 || !isfinite(r0)) {   // nothing to solve (or nothing finite): d = 0
    ctl[IC_STOP] = 1;
    sc[IS_INVB] = 0.0;
    return;
  }
  ctl[IC_STOP] = 0;
  g[0] = r0;
  sc[IS_INVB] = 1.0 / r0;
}

// Arnoldi column j: h (projection coefficients), ||w|| before and after the
// sweeps; earlier rotations, the new one, the estimate and the stop test
// (no tolerance: estimate exactly 0, breakdown, or the last step)
__global__ void k_ad_givens(int j, int q, double brk, const double* __restrict__ h, double* __restrict__ H,
                            double* __restrict__ g, double* __restrict__ cs, double* __restrict__ sn,
                            double* __restrict__ sc, int* __restrict__ ctl) {
  if (ctl[IC_STOP]) return;
  const int ldh = q + 1;
  double* col = H + (long long)ldh * j;
  const double wn0 = sqrt(sc[IS_WN0]), hn = sqrt(sc[IS_HN]);
  bool finite_h = true;
  for (int i = 0; i <= j; ++i) {
    col[i] = h[i];
    finite_h = finite_h && isfinite(h[i]);
  }
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i + 1] = -sn[i] * a + cs[i] * b;
    col[i] = cs[i] * a + sn[i] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double d = hypot(a, b);
  if (d == 0.0 || !isfinite(d) || !finite_h) {
    ctl[IC_STOP] = 1 + TG_NONFINITE;   // column j unusable
    return;
  }
  cs[j] = a / d;
  sn[j] = b / d;
  col[j] = d;
  col[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  ctl[IC_JDONE] = j + 1;
  const double est = fabs(g[j + 1]) / sc[IS_BNORM];
  if (est <= 0.0) ctl[IC_STOP] = 1 + TG_PROJ_CONVERGED;
  else if (hn <= brk * wn0) ctl[IC_STOP] = 1 + TG_BREAKDOWN;
  else if (j + 1 >= q) ctl[IC_STOP] = 1 + TG_MAXIT;
  sc[IS_INV] = 1.0 / hn;
}

// y = R^-1 g over the columns done
__global__ void k_ad_lsq(const double* __restrict__ H, int q, const double* __restrict__ g,
                         const int* __restrict__ ctl, double* __restrict__ y) {
  const int ldh = q + 1, jd = ctl[IC_JDONE];
  for (int i = jd - 1; i >= 0; --i) {
    double s = g[i];
    for (int k = i + 1; k < jd; ++k) s -= H[i + (long long)ldh * k] * y[k];
    y[i] = s / H[i + (long long)ldh * i];
  }
}

// out = *alpha * x, skipped once the inner iteration stopped
__global__ __launch_bounds__(AD_BLOCK) void k_ad_scale_dev(const double* __restrict__ x, const double* __restrict__ alpha,
                                                           const int* __restrict__ ctl, double* __restrict__ out,
                                                           long long n) {
  if (ctl[IC_STOP]) return;
  const double a = *alpha;
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK)
    out[i] = a * x[i];
}

// w = sum_{q < ctl[IC_JDONE]} c[q] V_q
__global__ __launch_bounds__(AD_BLOCK) void k_ad_combine_dev(const double* __restrict__ V, long long ld,
                                                             const int* __restrict__ ctl,
                                                             const double* __restrict__ c, double* __restrict__ w,
                                                             long long n) {
  __shared__ double sc[AD_MAXV];
  const int nv = ctl[IC_JDONE];
  for (int q = threadIdx.x; q < nv; q += AD_BLOCK) sc[q] = c[q];
  __syncthreads();
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK) {
    double s = 0.0;
    for (int q = 0; q < nv; ++q) s += sc[q] * V[(long long)q * ld + i];
    w[i] = s;
  }
}

// keep the correction iff ||s - K d|| < ||s||: z += d, and the decision in
// sc[IS_ACC]
__global__ __launch_bounds__(AD_BLOCK) void k_ad_accept(double* __restrict__ z, const double* __restrict__ d,
                                                        double* __restrict__ sc, long long n) {
  const bool ok = sqrt(sc[IS_R1SQ]) < sqrt(sc[IS_R0SQ]);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[IS_ACC] = ok ? 1.0 : 0.0;
  if (!ok) return;
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK)
    z[i] += d[i];
}

__global__ __launch_bounds__(AD_BLOCK) void k_ad_to32(const double* __restrict__ a, float* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK)
    b[i] = (float)a[i];
}
__global__ __launch_bounds__(AD_BLOCK) void k_ad_to64(const float* __restrict__ a, double* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK)
    b[i] = (double)a[i];
}

// Workspace of one call: outer basis (m + 1) + m vectors, inner basis
// (q + 1) + q vectors, four work vectors, two float vectors, partials and
// small device arrays.
struct Layout {
  long long n = 0, ld = 0;
  int m = 0, q = 0, nb = 0;
  size_t oV = 0, oZ = 0, iV = 0, iZ = 0, wv = 0, f32 = 0, part = 0, small = 0, ist = 0, total = 0;
  void init(const tg_grid* g, int restart, int inner) {
    n = g->lv[0].n_dof;
    ld = ld_of(n);
    m = restart;
    q = inner;
    nb = nblk_dots(n);
    const size_t vb = (size_t)ld * sizeof(double);
    size_t o = 0;
    oV = o; o += (size_t)(m > 0 ? m + 1 : 0) * vb;
    oZ = o; o += (size_t)m * vb;
    iV = o; o += (size_t)(q > 0 ? q + 1 : 0) * vb;
    iZ = o; o += (size_t)q * vb;
    wv = o; o += 4 * vb;
    f32 = o; o += 2 * al((size_t)n * sizeof(float));
    part = o; o += al((size_t)nb * AD_MAXV * sizeof(double));
    small = o; o += al(4 * AD_MAXV * sizeof(double));
    // inner state: Hessenberg (q + 1) x q, g, cs, sn, scalars, control ints
    ist = o; o += al(((size_t)(q + 1) * q + (q + 1) + 2 * q + IS_N) * sizeof(double) + IC_N * sizeof(int));
    total = o;
  }
};

struct Ctx {
  tg_grid* g;
  hipStream_t s;
  int prec;
  Layout L;
  char* base;
  double* vec(size_t off, int j) const { return (double*)(base + off) + (long long)j * L.ld; }
  double* W(int i) const { return vec(L.wv, i); }   // 0: w, 1: r / s, 2: t, 3: d
  float* r32() const { return (float*)(base + L.f32); }
  float* z32() const { return (float*)(base + L.f32 + al((size_t)L.n * sizeof(float))); }
  double* part() const { return (double*)(base + L.part); }
  double* tmp() const { return (double*)(base + L.small); }
  double* h() const { return tmp() + AD_MAXV; }
  double* coef() const { return tmp() + 2 * AD_MAXV; }
  double* scal() const { return tmp() + 3 * AD_MAXV; }   // ||w||^2 before and after orthogonalization
  // inner state
  double* iH() const { return (double*)(base + L.ist); }
  double* ig() const { return iH() + (size_t)(L.q + 1) * L.q; }
  double* ics() const { return ig() + L.q + 1; }
  double* isn() const { return ics() + L.q; }
  double* isc() const { return isn() + L.q; }
  int* ictl() const { return (int*)(isc() + IS_N); }
  bool flag_pending = false;   // a decision of M waits in isc()[IS_ACC]
  std::vector<int> accepted;
  // true-residual checkpoints of the outer iteration (every cp_every steps)
  struct Checkpoint {
    int k;
    double proj, eta;
  };
  int cp_every = 0;
  std::vector<Checkpoint> cps;
};

// out (default tmp) = V^T w over nv basis vectors; h = out or h += out (h
// may be NULL); self_out (may be NULL) = w^T w from the same pass
int dots(Ctx& c, const double* V, int nv, const double* w, double* h, int acc, double* out = nullptr,
         double* self_out = nullptr) {
  const int ws = self_out ? 1 : 0;
  dim3 grid(c.L.nb, (nv + ws + AD_QG - 1) / AD_QG);
  k_ad_dots<<<grid, AD_BLOCK, 0, c.s>>>(V, c.L.ld, nv, ws, w, c.L.n, c.part());
  TG_HIP(hipGetLastError());
  k_ad_sum<<<nv + ws, 64, 0, c.s>>>(c.part(), c.L.nb, nv, out ? out : c.tmp(), h, acc, self_out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

// w -= V coef (nv vectors), then *norm2_out = w^T w
int update_norm(Ctx& c, const double* V, int nv, const double* coef_d, double* w, double* norm2_out) {
  const int nb = nblk(c.L.n);
  k_ad_update_norm<<<nb, AD_BLOCK, 0, c.s>>>(V, c.L.ld, nv, coef_d, w, c.L.n, c.part());
  TG_HIP(hipGetLastError());
  k_ad_sum<<<1, 64, 0, c.s>>>(c.part(), nb, 0, nullptr, nullptr, 0, norm2_out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int norm(Ctx& c, const double* w, double* out) {
  int rc = dots(c, w, 1, w, nullptr, 0);
  if (rc) return rc;
  double v = 0.0;
  TG_HIP(hipMemcpyAsync(&v, c.tmp(), sizeof(double), hipMemcpyDeviceToHost, c.s));
  TG_HIP(hipStreamSynchronize(c.s));
  *out = std::sqrt(v);
  return TG_OK;
}

int axpby(Ctx& c, double a, const double* x, double b, const double* y, double* out) {
  k_ad_axpby<<<nblk(c.L.n), AD_BLOCK, 0, c.s>>>(a, x, b, y, out, c.L.n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int update(Ctx& c, const double* V, int nv, const double* coef_d, double sgn, double* w) {
  k_ad_update<<<nblk(c.L.n), AD_BLOCK, 0, c.s>>>(V, c.L.ld, nv, coef_d, sgn, w, c.L.n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int applyK(Ctx& c, const double* x, double* y) { return tg_apply_K(c.g, x, y, TG_F64, c.s); }

int jacobi(Ctx& c, const double* r, double* z) {
  k_ad_jacobi<<<nblk(c.g->lv[0].n_nodes), AD_BLOCK, 0, c.s>>>(c.g->desc.lv[0].Dinv64, r, z, c.g->lv[0].n_nodes,
                                                             c.g->nx + 1);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int vcycle(Ctx& c, const double* r, double* z) {
  if (c.prec == TG_F64) return tg_vcycle(c.g, r, z, TG_F64, c.s);
  k_ad_to32<<<nblk(c.L.n), AD_BLOCK, 0, c.s>>>(r, c.r32(), c.L.n);
  TG_HIP(hipGetLastError());
  const int rc = tg_vcycle(c.g, c.r32(), c.z32(), c.prec, c.s);
  if (rc) return rc;
  k_ad_to64<<<nblk(c.L.n), AD_BLOCK, 0, c.s>>>(c.z32(), z, c.L.n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

struct Krylov {
  double* V;
  double* Z;
  int m;
};

struct Outcome {
  std::vector<double> hist;
  int outcome = TG_PROJ_CONVERGED;
  int iters = 0;
};

// y = R^-1 g over the first jdone columns of the rotated Hessenberg
std::vector<double> lsq(const std::vector<double>& H, int ldh, const std::vector<double>& g, int jdone) {
  std::vector<double> y(jdone, 0.0);
  for (int i = jdone - 1; i >= 0; --i) {
    double s = g[i];
    for (int k = i + 1; k < jdone; ++k) s -= H[i + (size_t)ldh * k] * y[k];
    y[i] = s / H[i + (size_t)ldh * i];
  }
  return y;
}

// Right-preconditioned flexible GMRES on K x = b from x = 0 (Sec. 3.5) with
// the history semantics of the library's solver: hist[0] = 1, the true
// residual at every restart, the Givens estimate |g_{j+1}| / ||b|| inside a
// cycle; stop on estimate <= tol, breakdown, the iteration cap or a
// non-finite value.  CGS with `passes` sweeps (2 = CGS2 in place).
int fgmres(Ctx& c, const Krylov& K, const double* b, double* x, int max_iters, double tol, int passes, double brk,
           const std::function<int(const double*, double*)>& M, Outcome& out) {
  int rc;
  double* w = c.W(0);
  double* r = c.W(1);
  out = Outcome();
  TG_HIP(hipMemsetAsync(x, 0, sizeof(double) * c.L.n, c.s));
  double bnorm;
  if ((rc = norm(c, b, &bnorm))) return rc;
  out.hist.push_back(1.0);
  if (bnorm == 0.0) {
    out.hist[0] = 0.0;
    return TG_OK;
  }
  const int m = K.m, ldh = m + 1;
  std::vector<double> H((size_t)ldh * m), cs(m), sn(m), g(m + 1), hcol(AD_MAXV + 1);
  int k = 0;
  for (;;) {
    if (k > 0) {
      if ((rc = applyK(c, x, w))) return rc;
      if ((rc = axpby(c, 1.0, b, -1.0, w, r))) return rc;
    } else {
      TG_HIP(hipMemcpyAsync(r, b, sizeof(double) * c.L.n, hipMemcpyDeviceToDevice, c.s));
    }
    double beta;
    if ((rc = norm(c, r, &beta))) return rc;
    if (k > 0) out.hist[k] = beta / bnorm;
    out.iters = k;
    if (!std::isfinite(beta)) { out.outcome = TG_NONFINITE; return TG_OK; }
    if (beta / bnorm <= tol) { out.outcome = TG_PROJ_CONVERGED; return TG_OK; }
    if (k >= max_iters) { out.outcome = TG_MAXIT; return TG_OK; }
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    if ((rc = axpby(c, 1.0 / beta, r, 0.0, nullptr, K.V))) return rc;
    g[0] = beta;
    int stop = -1, jdone = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = K.V + (long long)j * c.L.ld;
      double* zj = K.Z + (long long)j * c.L.ld;
      if ((rc = M(vj, zj))) return rc;
      if ((rc = applyK(c, zj, w))) return rc;
      // ||w||^2 rides on the first sweep's dots, ||w||^2 after the last
      // sweep on its update
      for (int pass = 0; pass < passes; ++pass) {
        if ((rc = dots(c, K.V, j + 1, w, c.h(), pass > 0, nullptr, pass == 0 ? c.scal() : nullptr))) return rc;
        if (pass + 1 < passes) {
          if ((rc = update(c, K.V, j + 1, c.tmp(), -1.0, w))) return rc;
        } else if ((rc = update_norm(c, K.V, j + 1, c.tmp(), w, c.scal() + 1))) {
          return rc;
        }
      }
      double sq[2], acc = 0.0;
      TG_HIP(hipMemcpyAsync(hcol.data(), c.h(), sizeof(double) * (j + 1), hipMemcpyDeviceToHost, c.s));
      TG_HIP(hipMemcpyAsync(sq, c.scal(), sizeof(sq), hipMemcpyDeviceToHost, c.s));
      if (c.flag_pending) TG_HIP(hipMemcpyAsync(&acc, c.isc() + IS_ACC, sizeof(double), hipMemcpyDeviceToHost, c.s));
      TG_HIP(hipStreamSynchronize(c.s));
      if (c.flag_pending) {
        c.accepted.push_back(acc != 0.0 ? 1 : 0);
        c.flag_pending = false;
      }
      const double wnorm0 = std::sqrt(sq[0]), hn = std::sqrt(sq[1]);
      bool finite_h = true;
      for (int i = 0; i <= j; ++i) {
        H[i + (size_t)ldh * j] = hcol[i];
        finite_h = finite_h && std::isfinite(hcol[i]);
      }
      H[j + 1 + (size_t)ldh * j] = hn;
      for (int i = 0; i < j; ++i) {
        const double a = H[i + (size_t)ldh * j], bb = H[i + 1 + (size_t)ldh * j];
        H[i + 1 + (size_t)ldh * j] = -sn[i] * a + cs[i] * bb;
        H[i + (size_t)ldh * j] = cs[i] * a + sn[i] * bb;
      }
      const double a = H[j + (size_t)ldh * j], bb = H[j + 1 + (size_t)ldh * j];
      const double d = std::hypot(a, bb);
      if (d == 0.0 || !std::isfinite(d) || !finite_h) {
        stop = TG_NONFINITE;
        jdone = j;
        break;
      }
      cs[j] = a / d;
      sn[j] = bb / d;
      H[j + (size_t)ldh * j] = d;
      H[j + 1 + (size_t)ldh * j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++k;
      jdone = j + 1;
      const double est = std::fabs(g[j + 1]) / bnorm;
      out.hist.push_back(est);
      if (c.cp_every > 0 && k % c.cp_every == 0) {
        // recomputed residual of x_k = x + Z y_k, y_k over the columns so far;
        // the iteration itself is unchanged (W(2), W(3) are free between
        // applications of M)
        const std::vector<double> y = lsq(H, ldh, g, jdone);
        double* xk = c.W(3);
        double* t = c.W(2);
        TG_HIP(hipMemcpyAsync(c.coef(), y.data(), sizeof(double) * jdone, hipMemcpyHostToDevice, c.s));
        TG_HIP(hipMemcpyAsync(xk, x, sizeof(double) * c.L.n, hipMemcpyDeviceToDevice, c.s));
        if ((rc = update(c, K.Z, jdone, c.coef(), 1.0, xk))) return rc;
        if ((rc = applyK(c, xk, t))) return rc;
        if ((rc = axpby(c, 1.0, b, -1.0, t, t))) return rc;
        double rn;
        if ((rc = norm(c, t, &rn))) return rc;   // synchronizes: y is no longer read
        c.cps.push_back({k, est, rn / bnorm});
      }
      if (est <= tol) stop = TG_PROJ_CONVERGED;
      else if (hn <= brk * wnorm0) stop = TG_BREAKDOWN;
      else if (k >= max_iters) stop = TG_MAXIT;
      if (stop >= 0) break;
      if ((rc = axpby(c, 1.0 / hn, w, 0.0, nullptr, K.V + (long long)(j + 1) * c.L.ld))) return rc;
    }
    if (jdone > 0) {
      const std::vector<double> y = lsq(H, ldh, g, jdone);
      TG_HIP(hipMemcpyAsync(c.coef(), y.data(), sizeof(double) * jdone, hipMemcpyHostToDevice, c.s));
      if ((rc = update(c, K.Z, jdone, c.coef(), 1.0, x))) return rc;
      TG_HIP(hipStreamSynchronize(c.s));   // y lives on the host stack
    }
    if (stop >= 0) {
      out.outcome = stop;
      out.iters = k;
      return TG_OK;
    }
  }
}

// z = M(v): the V-cycle, then the accepted-or-rejected fine-level correction.
// The inner GMRES (restart = steps = q, CGS2, no tolerance) runs a fixed
// launch sequence whose scalar work and stop test live on the device; steps
// after a stop compute into columns that are never combined.  The decision
// is left in isc()[IS_ACC] (flag_pending), read with the caller's next
// synchronization.
int adaptive_apply(Ctx& c, const double* v, double* z) {
  int rc;
  if ((rc = vcycle(c, v, z))) return rc;
  c.flag_pending = true;
  if (c.L.q <= 0) {
    TG_HIP(hipMemsetAsync(c.isc() + IS_ACC, 0, sizeof(double), c.s));   // 0.0: nothing to keep
    return TG_OK;
  }
  const int q = c.L.q;
  const long long n = c.L.n;
  double* w = c.W(0);
  double* s = c.W(1);
  double* t = c.W(2);
  double* d = c.W(3);
  double* Vi = c.vec(c.L.iV, 0);
  double* Zi = c.vec(c.L.iZ, 0);
  double* sc = c.isc();
  int* ctl = c.ictl();
  const int nb = nblk(n);
  if ((rc = applyK(c, z, t))) return rc;
  if ((rc = axpby(c, 1.0, v, -1.0, t, s))) return rc;
  if ((rc = dots(c, s, 1, s, nullptr, 0, sc + IS_R0SQ))) return rc;
  k_ad_inner_init<<<1, 1, 0, c.s>>>(sc, ctl, c.ig());
  TG_HIP(hipGetLastError());
  k_ad_scale_dev<<<nb, AD_BLOCK, 0, c.s>>>(s, sc + IS_INVB, ctl, Vi, n);
  TG_HIP(hipGetLastError());
  for (int j = 0; j < q; ++j) {
    double* vj = Vi + (long long)j * c.L.ld;
    double* zj = Zi + (long long)j * c.L.ld;
    if ((rc = jacobi(c, vj, zj))) return rc;
    if ((rc = applyK(c, zj, w))) return rc;
    if ((rc = dots(c, Vi, j + 1, w, c.h(), 0, nullptr, sc + IS_WN0))) return rc;
    if ((rc = update(c, Vi, j + 1, c.tmp(), -1.0, w))) return rc;
    if ((rc = dots(c, Vi, j + 1, w, c.h(), 1))) return rc;
    if ((rc = update_norm(c, Vi, j + 1, c.tmp(), w, sc + IS_HN))) return rc;
    k_ad_givens<<<1, 1, 0, c.s>>>(j, q, 1e-14, c.h(), c.iH(), c.ig(), c.ics(), c.isn(), sc, ctl);
    TG_HIP(hipGetLastError());
    if (j + 1 < q) {
      k_ad_scale_dev<<<nb, AD_BLOCK, 0, c.s>>>(w, sc + IS_INV, ctl, Vi + (long long)(j + 1) * c.L.ld, n);
      TG_HIP(hipGetLastError());
    }
  }
  k_ad_lsq<<<1, 1, 0, c.s>>>(c.iH(), q, c.ig(), ctl, c.coef());
  TG_HIP(hipGetLastError());
  k_ad_combine_dev<<<nb, AD_BLOCK, 0, c.s>>>(Zi, c.L.ld, ctl, c.coef(), d, n);
  TG_HIP(hipGetLastError());
  if ((rc = applyK(c, d, t))) return rc;
  if ((rc = axpby(c, 1.0, s, -1.0, t, t))) return rc;
  if ((rc = dots(c, t, 1, t, nullptr, 0, sc + IS_R1SQ))) return rc;
  k_ad_accept<<<nb, AD_BLOCK, 0, c.s>>>(z, d, sc, n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int check_common(tg_grid* g, int prec, int restart, int inner, void* ws_d, size_t ws_bytes, Layout& L) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!g->density_set) return fail(TG_ESTATE, "set_density first");
  if (!ws_d) return fail(TG_EINVAL, "NULL workspace");
  if (prec < TG_F64 || prec > TG_BF16X3MFMA) return fail(TG_EINVAL, "unknown precision");
  if (restart < 0 || restart > TG_AD_MAX_RESTART || inner < 0 || inner > TG_AD_MAX_RESTART)
    return fail(TG_EINVAL, "restart and inner steps must lie in [0, TG_AD_MAX_RESTART]");
  L.init(g, restart, inner);
  if (ws_bytes < L.total) return fail(TG_EWORKSPACE, "adaptive workspace too small");
  return TG_OK;
}

}  // namespace

static int adaptive_solve_impl(tg_grid* g, const double* f_d, double* u_d, const tg_solver_opts* o, int inner_steps,
                        int every, int cap, void* ws_d, size_t ws_bytes, tg_solve_result* res, double* hist_h,
                        int* accepted_h, int* n_applied_h, int* k_h, double* proj_h, double* true_h, int* n_h,
                        void* stream) {
  if (!f_d || !u_d || !o || !res) return fail(TG_EINVAL, "NULL argument");
  if (o->restart < 1) return fail(TG_EINVAL, "restart must be >= 1");
  if (o->max_iters < 0 || !(o->tol >= 0.0)) return fail(TG_EINVAL, "need max_iters >= 0 and tol >= 0");
  if (o->cgs_passes < 1 || o->cgs_passes > 3) return fail(TG_EINVAL, "cgs_passes must be 1, 2 or 3");
  Layout L;
  int rc = check_common(g, o->prec, o->restart, inner_steps, ws_d, ws_bytes, L);
  if (rc) return rc;
  Ctx c{g, (hipStream_t)stream, o->prec, L, (char*)ws_d, {}};
  c.cp_every = every;
  Krylov outer{c.vec(L.oV, 0), c.vec(L.oZ, 0), L.m};
  Outcome out;
  auto M = [&c](const double* v, double* z) { return adaptive_apply(c, v, z); };
  if ((rc = fgmres(c, outer, f_d, u_d, o->max_iters, o->tol, o->cgs_passes == 1 ? 1 : 2, o->breakdown, M, out)))
    return rc;
  TG_HIP(hipStreamSynchronize(c.s));
  res->iterations = out.iters;
  res->outcome = out.outcome;
  res->proj_eta = out.hist.back();
  res->true_eta = -1.0;
  if (hist_h) std::memcpy(hist_h, out.hist.data(), sizeof(double) * out.hist.size());
  const int na = (int)std::min<size_t>(c.accepted.size(), (size_t)o->max_iters + 1);
  if (accepted_h) std::copy(c.accepted.begin(), c.accepted.begin() + na, accepted_h);
  if (n_applied_h) *n_applied_h = (int)c.accepted.size();
  if (n_h) {
    const int nc = (int)std::min<size_t>(c.cps.size(), (size_t)cap);
    for (int i = 0; i < nc; ++i) {
      k_h[i] = c.cps[i].k;
      proj_h[i] = c.cps[i].proj;
      true_h[i] = c.cps[i].eta;
    }
    *n_h = nc;
  }
  return TG_OK;
}

}  // namespace tg

using namespace tg;

extern "C" {

int tg_adaptive_workspace_bytes(const tg_grid* g, int restart, int inner_steps, size_t* bytes) {
  if (!g || !bytes) return fail(TG_EINVAL, "NULL argument");
  if (restart < 0 || restart > TG_AD_MAX_RESTART || inner_steps < 0 || inner_steps > TG_AD_MAX_RESTART)
    return fail(TG_EINVAL, "restart and inner steps must lie in [0, TG_AD_MAX_RESTART]");
  Layout L;
  L.init(g, restart, inner_steps);
  *bytes = L.total;
  return TG_OK;
}

int tg_adaptive_precondition(tg_grid* g, const double* v_d, double* z_d, int prec, int inner_steps, void* ws_d,
                             size_t ws_bytes, int* accepted_h, void* stream) {
  if (!v_d || !z_d) return fail(TG_EINVAL, "NULL vector");
  Layout L;
  int rc = check_common(g, prec, 0, inner_steps, ws_d, ws_bytes, L);
  if (rc) return rc;
  Ctx c{g, (hipStream_t)stream, prec, L, (char*)ws_d, {}};
  if ((rc = adaptive_apply(c, v_d, z_d))) return rc;
  double acc = 0.0;
  TG_HIP(hipMemcpyAsync(&acc, c.isc() + IS_ACC, sizeof(double), hipMemcpyDeviceToHost, c.s));
  TG_HIP(hipStreamSynchronize(c.s));
  if (accepted_h) *accepted_h = acc != 0.0 ? 1 : 0;
  return TG_OK;
}

int tg_adaptive_solve(tg_grid* g, const double* f_d, double* u_d, const tg_solver_opts* o, int inner_steps,
                      void* ws_d, size_t ws_bytes, tg_solve_result* res, double* hist_h, int* accepted_h,
                      int* n_applied_h, void* stream) {
  return tg::adaptive_solve_impl(g, f_d, u_d, o, inner_steps, 0, 0, ws_d, ws_bytes, res, hist_h, accepted_h,
                                 n_applied_h, nullptr, nullptr, nullptr, nullptr, stream);
}

int tg_adaptive_checkpoints(tg_grid* g, const double* f_d, double* u_d, const tg_solver_opts* o, int inner_steps,
                            int every, int cap, void* ws_d, size_t ws_bytes, tg_solve_result* res, int* k_h,
                            double* proj_h, double* true_h, int* n_h, void* stream) {
  if (every < 1 || cap < 0) return fail(TG_EINVAL, "need every >= 1 and cap >= 0");
  if (cap > 0 && (!k_h || !proj_h || !true_h)) return fail(TG_EINVAL, "NULL checkpoint array");
  if (!n_h) return fail(TG_EINVAL, "NULL argument");
  return tg::adaptive_solve_impl(g, f_d, u_d, o, inner_steps, every, cap, ws_d, ws_bytes, res, nullptr, nullptr,
                                 nullptr, k_h, proj_h, true_h, n_h, stream);
}

}  // extern "C"
