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

// ---- kernels of the full adaptive stack (Chebyshev smoothing, line-searched
// coarse correction)

// scalars of the stack: the log of one application first (read by the host)
enum { ST_ALPHA = 0, ST_RATIO = 1, ST_OK = 2, ST_RKD = 3, ST_KK = 4, ST_TT = 5, ST_RR = 6, ST_PW = 7, ST_N = 16 };

// start vector of the power iteration: DOF d of the level's full numbering
// (x-fastest nodes, three components) gets ((d + 1) * 0x9E3779B1 mod 2^32) /
// 2^32 - 0.5, exact in FP64; the clamped nodes get 0
__global__ __launch_bounds__(AD_BLOCK) void k_st_hash(double* __restrict__ v, long long n_nodes, int NX) {
  for (long long d = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; d < 3 * n_nodes;
       d += (long long)gridDim.x * AD_BLOCK) {
    const unsigned int h = (unsigned int)((unsigned long long)(d + 1) * 0x9E3779B1ull);
    v[d] = ((d / 3) % NX == 0) ? 0.0 : (double)h / 4294967296.0 - 0.5;
  }
}

// out = x / sqrt(*ss)
__global__ __launch_bounds__(AD_BLOCK) void k_st_div_norm(const double* __restrict__ x, const double* __restrict__ ss,
                                                          double* __restrict__ out, long long n) {
  const double nr = sqrt(*ss);
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK)
    out[i] = x[i] / nr;
}

__global__ void k_st_sqrt(const double* __restrict__ ss, double* __restrict__ out) { *out = sqrt(*ss); }

// x = omega D^-1 b node by node at one level (D the 3 x 3 diagonal block of
// K at the node); the clamped nodes get 0
__global__ __launch_bounds__(AD_BLOCK) void k_st_jacobi(const double* __restrict__ Dinv, const double* __restrict__ b,
                                                        double* __restrict__ x, double omega, long long n_nodes,
                                                        int NX) {
  for (long long v = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; v < n_nodes;
       v += (long long)gridDim.x * AD_BLOCK) {
    const double b0 = b[3 * v], b1 = b[3 * v + 1], b2 = b[3 * v + 2];
    const double* D = Dinv + 9 * v;
    const bool fixed = (v % NX) == 0;
    x[3 * v] = fixed ? 0.0 : omega * (D[0] * b0 + D[1] * b1 + D[2] * b2);
    x[3 * v + 1] = fixed ? 0.0 : omega * (D[3] * b0 + D[4] * b1 + D[5] * b2);
    x[3 * v + 2] = fixed ? 0.0 : omega * (D[6] * b0 + D[7] * b1 + D[8] * b2);
  }
}

// the momentum term of a Chebyshev step: y += beta (x - xp) (xp NULL: zero)
__global__ __launch_bounds__(AD_BLOCK) void k_st_cheb_fix(double* __restrict__ y, const double* __restrict__ x,
                                                          const double* __restrict__ xp, double beta, long long n) {
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK)
    y[i] += beta * (xp ? x[i] - xp[i] : x[i]);
}

// bc = P^T rf (full weighting, the transpose of the trilinear prolongation):
// coarse node (I, J, K) sums the fine nodes (2I + a, 2J + b, 2K + c),
// a, b, c in {-1, 0, 1}, weighted by 1/2 per nonzero offset; the clamped
// coarse nodes (I = 0) get 0
__global__ __launch_bounds__(AD_BLOCK) void k_st_restrict(const double* __restrict__ rf, double* __restrict__ bc,
                                                          int NXf, int NYf, int NZf, int NXc, int NYc, int NZc) {
  const long long nc = (long long)NXc * NYc * NZc;
  for (long long m = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; m < nc; m += (long long)gridDim.x * AD_BLOCK) {
    const int I = (int)(m % NXc);
    const long long t = m / NXc;
    const int J = (int)(t % NYc), K = (int)(t / NYc);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (I > 0) {
      for (int c = -1; c <= 1; ++c) {
        const int k = 2 * K + c;
        if (k < 0 || k >= NZf) continue;
        for (int b = -1; b <= 1; ++b) {
          const int j = 2 * J + b;
          if (j < 0 || j >= NYf) continue;
          for (int a = -1; a <= 1; ++a) {
            const int i = 2 * I + a;
            if (i < 0 || i >= NXf) continue;
            const double w = 1.0 / (double)(1 << ((a != 0) + (b != 0) + (c != 0)));
            const long long f = 3 * (i + (long long)NXf * (j + (long long)NYf * k));
            s0 += w * rf[f];
            s1 += w * rf[f + 1];
            s2 += w * rf[f + 2];
          }
        }
      }
    }
    bc[3 * m] = s0;
    bc[3 * m + 1] = s1;
    bc[3 * m + 2] = s2;
  }
}

// line search: alpha = (r . Kd) / (Kd . Kd), 0 when Kd = 0
__global__ void k_st_alpha(double* __restrict__ st) {
  st[ST_ALPHA] = st[ST_KK] > 0.0 ? st[ST_RKD] / st[ST_KK] : 0.0;
}

// t = r - alpha Kd
__global__ __launch_bounds__(AD_BLOCK) void k_st_axmy(const double* __restrict__ r, const double* __restrict__ Kd,
                                                      const double* __restrict__ st, double* __restrict__ t,
                                                      long long n) {
  const double a = st[ST_ALPHA];
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK)
    t[i] = r[i] - a * Kd[i];
}

// ratio = ||r - alpha Kd|| / ||r|| (1 when r = 0); the correction is kept,
// x += alpha d, iff ratio <= theta (the acceptance ratio)
__global__ __launch_bounds__(AD_BLOCK) void k_st_accept(double* __restrict__ st, double theta, double* __restrict__ x,
                                                        const double* __restrict__ d, long long n) {
  const double nr = sqrt(st[ST_RR]);
  const double ratio = nr > 0.0 ? sqrt(st[ST_TT]) / nr : 1.0;
  const bool ok = ratio <= theta;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st[ST_RATIO] = ratio;
    st[ST_OK] = ok ? 1.0 : 0.0;
  }
  if (!ok) return;
  const double a = st[ST_ALPHA];
  for (long long i = (long long)blockIdx.x * AD_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * AD_BLOCK)
    x[i] += a * d[i];
}

size_t inner_state_bytes(int q) {
  // Hessenberg (q + 1) x q, g, cs, sn, scalars, control ints
  return al(((size_t)(q + 1) * q + (q + 1) + 2 * q + IS_N) * sizeof(double) + IC_N * sizeof(int));
}

// Workspace of one call: outer basis (m + 1) + m vectors, inner basis
// (q + 1) + q vectors, four work vectors, two float vectors, partials and
// small device arrays.  The full stack adds six fine vectors, the level-1
// Krylov basis (cs + 1) + cs vectors and three level-1 work vectors, the
// level-1 inner state and the stack's scalars.
struct Layout {
  long long n = 0, ld = 0, n1 = 0, ld1 = 0;
  int m = 0, q = 0, nb = 0, cs = 0;
  bool stack = false;
  size_t oV = 0, oZ = 0, iV = 0, iZ = 0, wv = 0, f32 = 0, part = 0, small = 0, ist = 0;
  size_t s0 = 0, c1V = 0, c1Z = 0, c1x = 0, cist = 0, stk = 0, total = 0;
  void init(const tg_grid* g, int restart, int inner, bool with_stack = false, int coarse = 0) {
    n = g->lv[0].n_dof;
    ld = ld_of(n);
    m = restart;
    q = inner;
    nb = nblk_dots(n);
    stack = with_stack;
    cs = with_stack ? coarse : 0;
    n1 = (with_stack && g->nlev > 1) ? 3LL * g->lv[1].n_nodes : 0;
    ld1 = ld_of(n1);
    const size_t vb = (size_t)ld * sizeof(double), vb1 = (size_t)ld1 * sizeof(double);
    size_t o = 0;
    oV = o; o += (size_t)(m > 0 ? m + 1 : 0) * vb;
    oZ = o; o += (size_t)m * vb;
    iV = o; o += (size_t)(q > 0 ? q + 1 : 0) * vb;
    iZ = o; o += (size_t)q * vb;
    wv = o; o += 4 * vb;
    f32 = o; o += 2 * al((size_t)n * sizeof(float));
    part = o; o += al((size_t)nb * AD_MAXV * sizeof(double));
    small = o; o += al(4 * AD_MAXV * sizeof(double));
    ist = o; o += inner_state_bytes(q);
    if (stack) {
      s0 = o; o += 6 * vb;
      c1V = o; o += (size_t)(cs > 0 ? cs + 1 : 0) * vb1;
      c1Z = o; o += (size_t)cs * vb1;
      c1x = o; o += 3 * vb1;
      cist = o; o += inner_state_bytes(cs);
      stk = o; o += al((ST_N + TG_MAXLEV) * sizeof(double));
    }
    total = o;
  }
};

// One inner GMRES: its basis, Hessenberg and device scalars.
struct Inner {
  double* V;
  double* Z;
  long long ld, n;
  int q;
  double* H;
  double* g;
  double* cs;
  double* sn;
  double* sc;
  int* ctl;
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
  // an inner state at byte offset off with q columns, basis V (q + 1) and Z (q)
  Inner inner_at(size_t off, int q, double* V, double* Z, long long ld_, long long n_) const {
    Inner S;
    S.V = V;
    S.Z = Z;
    S.ld = ld_;
    S.n = n_;
    S.q = q;
    S.H = (double*)(base + off);
    S.g = S.H + (size_t)(q + 1) * q;
    S.cs = S.g + q + 1;
    S.sn = S.cs + q;
    S.sc = S.sn + q;
    S.ctl = (int*)(S.sc + IS_N);
    return S;
  }
  Inner fine_inner() const { return inner_at(L.ist, L.q, vec(L.iV, 0), vec(L.iZ, 0), L.ld, L.n); }
  Inner coarse_inner() const {
    return inner_at(L.cist, L.cs, (double*)(base + L.c1V), (double*)(base + L.c1Z), L.ld1, L.n1);
  }
  // stack vectors: fine S0(0..5), level-1 work C1(0..2), scalars, lambdas
  double* S0(int i) const { return vec(L.s0, i); }
  double* C1(int i) const { return (double*)(base + L.c1x) + (long long)i * L.ld1; }
  double* stk() const { return (double*)(base + L.stk); }
  double* lams_d() const { return stk() + ST_N; }
  bool flag_pending = false;   // a decision of M waits in isc()[IS_ACC]
  std::vector<int> accepted;
  // the full stack: options, lambda~ per level, one log entry per application
  bool stack = false;
  tg_stack_opts so{};
  double lam[TG_MAXLEV] = {};
  std::vector<tg_stack_log> slog;
  // true-residual checkpoints of the outer iteration (every cp_every steps)
  struct Checkpoint {
    int k;
    double proj, eta;
  };
  int cp_every = 0;
  std::vector<Checkpoint> cps;
};

// out (default tmp) = V^T w over nv basis vectors of n entries (leading
// dimension ld); h = out or h += out (h may be NULL); self_out (may be NULL)
// = w^T w from the same pass
int dots_n(Ctx& c, long long ld, long long n, const double* V, int nv, const double* w, double* h, int acc,
           double* out = nullptr, double* self_out = nullptr) {
  const int ws = self_out ? 1 : 0;
  const int nb = nblk_dots(n);
  dim3 grid(nb, (nv + ws + AD_QG - 1) / AD_QG);
  k_ad_dots<<<grid, AD_BLOCK, 0, c.s>>>(V, ld, nv, ws, w, n, c.part());
  TG_HIP(hipGetLastError());
  k_ad_sum<<<nv + ws, 64, 0, c.s>>>(c.part(), nb, nv, out ? out : c.tmp(), h, acc, self_out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}
int dots(Ctx& c, const double* V, int nv, const double* w, double* h, int acc, double* out = nullptr,
         double* self_out = nullptr) {
  return dots_n(c, c.L.ld, c.L.n, V, nv, w, h, acc, out, self_out);
}

// w -= V coef (nv vectors), then *norm2_out = w^T w
int update_norm_n(Ctx& c, long long ld, long long n, const double* V, int nv, const double* coef_d, double* w,
                  double* norm2_out) {
  const int nb = nblk(n);
  k_ad_update_norm<<<nb, AD_BLOCK, 0, c.s>>>(V, ld, nv, coef_d, w, n, c.part());
  TG_HIP(hipGetLastError());
  k_ad_sum<<<1, 64, 0, c.s>>>(c.part(), nb, 0, nullptr, nullptr, 0, norm2_out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}
int update_norm(Ctx& c, const double* V, int nv, const double* coef_d, double* w, double* norm2_out) {
  return update_norm_n(c, c.L.ld, c.L.n, V, nv, coef_d, w, norm2_out);
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

int update_n(Ctx& c, long long ld, long long n, const double* V, int nv, const double* coef_d, double sgn,
             double* w) {
  k_ad_update<<<nblk(n), AD_BLOCK, 0, c.s>>>(V, ld, nv, coef_d, sgn, w, n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}
int update(Ctx& c, const double* V, int nv, const double* coef_d, double sgn, double* w) {
  return update_n(c, c.L.ld, c.L.n, V, nv, coef_d, sgn, w);
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
      double sq[2], acc = 0.0, lg[3] = {0.0, 0.0, 0.0};
      TG_HIP(hipMemcpyAsync(hcol.data(), c.h(), sizeof(double) * (j + 1), hipMemcpyDeviceToHost, c.s));
      TG_HIP(hipMemcpyAsync(sq, c.scal(), sizeof(sq), hipMemcpyDeviceToHost, c.s));
      if (c.flag_pending) TG_HIP(hipMemcpyAsync(&acc, c.isc() + IS_ACC, sizeof(double), hipMemcpyDeviceToHost, c.s));
      if (c.flag_pending && c.stack) TG_HIP(hipMemcpyAsync(lg, c.stk(), sizeof(lg), hipMemcpyDeviceToHost, c.s));
      TG_HIP(hipStreamSynchronize(c.s));
      if (c.flag_pending) {
        c.accepted.push_back(acc != 0.0 ? 1 : 0);
        if (c.stack) c.slog.push_back({lg[ST_ALPHA], lg[ST_RATIO], lg[ST_OK] != 0.0 ? 1 : 0, acc != 0.0 ? 1 : 0});
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

// d = the iterate after S.q steps of right-preconditioned GMRES on A d = rhs
// from d = 0 (restart = steps = q, CGS2, no tolerance stop): a fixed launch
// sequence whose scalar work and stop test (breakdown, non-finite, estimate
// exactly 0) live on the device; steps after a stop compute into columns
// that are never combined.  w: a work vector of S.n entries.
template <class AF, class MF>
int inner_gmres(Ctx& c, const Inner& S, const double* rhs, double* w, double* d, AF&& A, MF&& M) {
  int rc;
  const int q = S.q;
  const long long n = S.n, ld = S.ld;
  const int nb = nblk(n);
  if ((rc = dots_n(c, ld, n, rhs, 1, rhs, nullptr, 0, S.sc + IS_R0SQ))) return rc;
  k_ad_inner_init<<<1, 1, 0, c.s>>>(S.sc, S.ctl, S.g);
  TG_HIP(hipGetLastError());
  k_ad_scale_dev<<<nb, AD_BLOCK, 0, c.s>>>(rhs, S.sc + IS_INVB, S.ctl, S.V, n);
  TG_HIP(hipGetLastError());
  for (int j = 0; j < q; ++j) {
    double* vj = S.V + (long long)j * ld;
    double* zj = S.Z + (long long)j * ld;
    if ((rc = M(vj, zj))) return rc;
    if ((rc = A(zj, w))) return rc;
    if ((rc = dots_n(c, ld, n, S.V, j + 1, w, c.h(), 0, nullptr, S.sc + IS_WN0))) return rc;
    if ((rc = update_n(c, ld, n, S.V, j + 1, c.tmp(), -1.0, w))) return rc;
    if ((rc = dots_n(c, ld, n, S.V, j + 1, w, c.h(), 1))) return rc;
    if ((rc = update_norm_n(c, ld, n, S.V, j + 1, c.tmp(), w, S.sc + IS_HN))) return rc;
    k_ad_givens<<<1, 1, 0, c.s>>>(j, q, 1e-14, c.h(), S.H, S.g, S.cs, S.sn, S.sc, S.ctl);
    TG_HIP(hipGetLastError());
    if (j + 1 < q) {
      k_ad_scale_dev<<<nb, AD_BLOCK, 0, c.s>>>(w, S.sc + IS_INV, S.ctl, S.V + (long long)(j + 1) * ld, n);
      TG_HIP(hipGetLastError());
    }
  }
  k_ad_lsq<<<1, 1, 0, c.s>>>(S.H, q, S.g, S.ctl, c.coef());
  TG_HIP(hipGetLastError());
  k_ad_combine_dev<<<nb, AD_BLOCK, 0, c.s>>>(S.Z, ld, S.ctl, c.coef(), d, n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

// The fine-level correction of z (Tab. solver-config): with s = v - K z, q
// inner GMRES steps on K d = s preconditioned by the node-block Jacobi
// operator; z += d iff ||s - K d|| < ||s||.  The decision is left in
// isc()[IS_ACC] (flag_pending), read with the caller's next synchronization.
int fine_correction(Ctx& c, const double* v, double* z) {
  int rc;
  c.flag_pending = true;
  if (c.L.q <= 0) {
    TG_HIP(hipMemsetAsync(c.isc() + IS_ACC, 0, sizeof(double), c.s));   // 0.0: nothing to keep
    return TG_OK;
  }
  double* s = c.W(1);
  double* t = c.W(2);
  double* d = c.W(3);
  double* sc = c.isc();
  if ((rc = applyK(c, z, t))) return rc;
  if ((rc = axpby(c, 1.0, v, -1.0, t, s))) return rc;
  rc = inner_gmres(c, c.fine_inner(), s, c.W(0), d, [&c](const double* x, double* y) { return applyK(c, x, y); },
                   [&c](const double* x, double* y) { return jacobi(c, x, y); });
  if (rc) return rc;
  if ((rc = applyK(c, d, t))) return rc;
  if ((rc = axpby(c, 1.0, s, -1.0, t, t))) return rc;
  if ((rc = dots(c, t, 1, t, nullptr, 0, sc + IS_R1SQ))) return rc;
  k_ad_accept<<<nblk(c.L.n), AD_BLOCK, 0, c.s>>>(z, d, sc, c.L.n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

// z = M(v): the V-cycle, then the accepted-or-rejected fine-level correction.
int adaptive_apply(Ctx& c, const double* v, double* z) {
  int rc;
  if ((rc = vcycle(c, v, z))) return rc;
  return fine_correction(c, v, z);
}

// ---- the full adaptive stack (Tab. solver-config; Sec. 3.5)
//
// One application z = M(v), all in FP64:
//   x  = Chebyshev iteration of degree nu_pre on K x = v from 0 (finest level);
//   r  = v - K x, b1 = P^T r;
//   e  = coarse_steps steps of GMRES (restart = steps) on K_1 e = b1 from 0,
//        right-preconditioned by the Chebyshev V-cycle of levels 1.. (one such
//        V-cycle if coarse_steps = 0, the direct solve if level 1 is the
//        coarsest);
//   d  = P e; alpha minimizes ||r - alpha K d||; x += alpha d iff
//        ||r - alpha K d|| <= theta ||r||;
//   z  = Chebyshev iteration of degree nu_post from x;
//   then the fine-level correction of z.
// The Chebyshev iteration at level l runs on [lo, hi] * lambda~_l, lambda~_l
// from power_iters power steps on D_l^-1 K_l from a hashed start vector.
// Every decision is taken on the device; the log (alpha, ratio, accepted) is
// read with the caller's next synchronization.

long long lvl_n(const Ctx& c, int l) { return 3LL * c.g->lv[l].n_nodes; }
double* pool64(const Ctx& c, int l, int slot) {
  return c.g->desc.lv[l].vec64 + (long long)slot * c.g->desc.lv[l].stride;
}

// (omega_k, beta_k), k < deg, of the three-term Chebyshev step
// x_{k+1} = x_k + omega_k D^-1 (b - K x_k) + beta_k (x_k - x_{k-1}) on the
// interval [lo lam, hi lam]: centre c, half-width h, sigma = c / h,
// rho_0 = 1 / sigma, rho_k = 1 / (2 sigma - rho_{k-1}); omega_0 = 1 / c,
// beta_0 = 0, omega_k = 2 rho_k / h, beta_k = rho_k rho_{k-1}
void cheb_coefs(double lam, int deg, double lo, double hi, double* om, double* be) {
  const double a = lo * lam, b = hi * lam;
  const double c = 0.5 * (a + b), h = 0.5 * (b - a);
  const double sigma = c / h;
  om[0] = 1.0 / c;
  be[0] = 0.0;
  double rho = 1.0 / sigma;
  for (int k = 1; k < deg; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    om[k] = 2.0 * rn / h;
    be[k] = rn * rho;
    rho = rn;
  }
}

int st_jacobi(Ctx& c, int l, const double* b, double* x, double om) {
  const long long nn = c.g->lv[l].n_nodes;
  k_st_jacobi<<<nblk(nn), AD_BLOCK, 0, c.s>>>(c.g->desc.lv[l].Dinv64, b, x, om, nn, c.g->desc.lv[l].NX);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

constexpr int ST_MAX_DEGREE = 16;

// Chebyshev iteration of degree deg at level l on K_l x = b from x0 (NULL:
// from zero).  The iterates rotate through rot[0..2] (distinct from b; x0 may
// be one of them); the last goes to out if out is non-NULL (distinct from b,
// x0 and rot), else it stays in rot.  *res = the result.
int cheb(Ctx& c, int l, const double* b, const double* x0, double* out, int deg, double* const* rot,
         const double** res) {
  int rc;
  double om[ST_MAX_DEGREE], be[ST_MAX_DEGREE];
  cheb_coefs(c.lam[l], deg, c.so.lo, c.so.hi, om, be);
  const long long n = lvl_n(c, l);
  const double* xc = x0;   // x_k
  const double* xp = x0;   // x_{k-1}
  for (int k = 0; k < deg; ++k) {
    double* dst = (k == deg - 1) ? out : nullptr;
    for (int i = 0; i < 3 && !dst; ++i)
      if (rot[i] != xc && rot[i] != xp) dst = rot[i];
    if (!xc) {
      if ((rc = st_jacobi(c, l, b, dst, om[0]))) return rc;   // x_1 = omega_0 D^-1 b
    } else {
      if ((rc = level_op64(c.g->self, l, LV_SMOOTH, xc, b, dst, om[k], c.s))) return rc;
      if (be[k] != 0.0) {
        k_st_cheb_fix<<<nblk(n), AD_BLOCK, 0, c.s>>>(dst, xc, xp, be[k], n);
        TG_HIP(hipGetLastError());
      }
    }
    xp = xc;
    xc = dst;
  }
  *res = xc;
  return TG_OK;
}

// The V-cycle with Chebyshev smoothing from level l >= 1 on K_l x = b (b an
// external vector or level l's slot C_B): result to out if non-NULL (distinct
// from b and level l's other slots), else left in one of level l's slots
// C_XA, C_XB, C_R; *res = the result.
int cheb_vcycle(Ctx& c, int l, const double* b, double* out, const double** res) {
  int rc;
  Batch* B = c.g->self;
  if (l == c.g->nlev - 1) {
    double* y = out ? out : pool64(c, l, C_XA);
    if ((rc = level_coarse64(B, l, b, y, c.s))) return rc;
    *res = y;
    return TG_OK;
  }
  double* rot[3] = {pool64(c, l, C_XA), pool64(c, l, C_XB), pool64(c, l, C_R)};
  const double* x;
  const double* e;
  if ((rc = cheb(c, l, b, nullptr, nullptr, c.so.nu_pre, rot, &x))) return rc;
  // the residual restricted straight into level l + 1's right-hand side
  if ((rc = level_restrict64(B, l, x, b, C_B, c.s))) return rc;
  if ((rc = cheb_vcycle(c, l + 1, pool64(c, l + 1, C_B), nullptr, &e))) return rc;
  if ((rc = level_prolong64(B, l, e, const_cast<double*>(x), c.s))) return rc;
  return cheb(c, l, b, x, out, c.so.nu_post, rot, res);
}

// lambda~ of every level above the coarsest into c.lam (synchronizes)
int stack_setup(Ctx& c) {
  int rc;
  Batch* B = c.g->self;
  double* st = c.stk();
  const int nl = c.g->nlev - 1;
  for (int l = 0; l < nl; ++l) {
    const long long n = lvl_n(c, l);
    double* v = l == 0 ? c.S0(0) : pool64(c, l, C_XA);
    double* t = l == 0 ? c.S0(1) : pool64(c, l, C_XB);
    double* w = l == 0 ? c.S0(2) : pool64(c, l, C_R);
    const int nb = nblk(n);
    k_st_hash<<<nb, AD_BLOCK, 0, c.s>>>(v, c.g->lv[l].n_nodes, c.g->desc.lv[l].NX);
    TG_HIP(hipGetLastError());
    if ((rc = dots_n(c, n, n, v, 1, v, nullptr, 0, st + ST_PW))) return rc;
    k_st_div_norm<<<nb, AD_BLOCK, 0, c.s>>>(v, st + ST_PW, v, n);
    TG_HIP(hipGetLastError());
    for (int it = 0; it < c.so.power_iters; ++it) {
      if ((rc = level_op64(B, l, LV_APPLY, v, nullptr, t, 0.0, c.s))) return rc;
      if ((rc = st_jacobi(c, l, t, w, 1.0))) return rc;
      if ((rc = dots_n(c, n, n, w, 1, w, nullptr, 0, st + ST_PW))) return rc;
      k_st_div_norm<<<nb, AD_BLOCK, 0, c.s>>>(w, st + ST_PW, v, n);
      TG_HIP(hipGetLastError());
    }
    k_st_sqrt<<<1, 1, 0, c.s>>>(st + ST_PW, c.lams_d() + l);
    TG_HIP(hipGetLastError());
  }
  TG_HIP(hipMemcpyAsync(c.lam, c.lams_d(), sizeof(double) * nl, hipMemcpyDeviceToHost, c.s));
  TG_HIP(hipStreamSynchronize(c.s));
  return TG_OK;
}

// z = M(v) of the full stack (v and z distinct, n_dof entries each)
int stack_apply(Ctx& c, const double* v, double* z) {
  int rc;
  Batch* B = c.g->self;
  const long long n = c.L.n;
  const int nb = nblk(n);
  double* rot[3] = {c.S0(0), c.S0(1), c.S0(2)};
  double* r = c.S0(3);
  double* dc = c.S0(4);
  double* Kd = c.S0(5);
  double* st = c.stk();
  const double* x;
  const double* xo;
  if ((rc = cheb(c, 0, v, nullptr, nullptr, c.so.nu_pre, rot, &x))) return rc;
  if ((rc = level_op64(B, 0, LV_RESID, x, v, r, 0.0, c.s))) return rc;
  // coarse right-hand side b1 = P^T r and the coarse correction e
  double* b1 = c.C1(0);
  double* e = c.C1(1);
  const LevelDesc& L0 = c.g->desc.lv[0];
  const LevelDesc& L1 = c.g->desc.lv[1];
  k_st_restrict<<<nblk(c.g->lv[1].n_nodes), AD_BLOCK, 0, c.s>>>(r, b1, L0.NX, L0.NY, L0.NZ, L1.NX, L1.NY, L1.NZ);
  TG_HIP(hipGetLastError());
  if (c.g->nlev == 2) {
    if ((rc = level_coarse64(B, 1, b1, e, c.s))) return rc;
  } else if (c.L.cs == 0) {
    if ((rc = cheb_vcycle(c, 1, b1, e, &xo))) return rc;
  } else {
    auto A1 = [&c, B](const double* a, double* y) { return level_op64(B, 1, LV_APPLY, a, nullptr, y, 0.0, c.s); };
    auto M1 = [&c](const double* a, double* y) {
      const double* res;
      return cheb_vcycle(c, 1, a, y, &res);
    };
    if ((rc = inner_gmres(c, c.coarse_inner(), b1, c.C1(2), e, A1, M1))) return rc;
  }
  // d = P e, K d, and the line search on the fine residual
  TG_HIP(hipMemsetAsync(dc, 0, sizeof(double) * n, c.s));
  if ((rc = level_prolong64(B, 0, e, dc, c.s))) return rc;
  if ((rc = level_op64(B, 0, LV_APPLY, dc, nullptr, Kd, 0.0, c.s))) return rc;
  if ((rc = dots(c, r, 1, Kd, nullptr, 0, st + ST_RKD, st + ST_KK))) return rc;
  k_st_alpha<<<1, 1, 0, c.s>>>(st);
  TG_HIP(hipGetLastError());
  k_st_axmy<<<nb, AD_BLOCK, 0, c.s>>>(r, Kd, st, c.W(2), n);
  TG_HIP(hipGetLastError());
  if ((rc = dots(c, c.W(2), 1, c.W(2), nullptr, 0, st + ST_TT))) return rc;
  if ((rc = dots(c, r, 1, r, nullptr, 0, st + ST_RR))) return rc;
  k_st_accept<<<nb, AD_BLOCK, 0, c.s>>>(st, c.so.theta, const_cast<double*>(x), dc, n);
  TG_HIP(hipGetLastError());
  if ((rc = cheb(c, 0, v, x, z, c.so.nu_post, rot, &xo))) return rc;
  return fine_correction(c, v, z);
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

int stack_check(tg_grid* g, const tg_stack_opts* so, int restart, void* ws_d, size_t ws_bytes, Layout& L) {
  if (!so) return fail(TG_EINVAL, "NULL stack options");
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!g->density_set) return fail(TG_ESTATE, "set_density first");
  if (!g->coarse_ok) return fail(TG_EINVAL, "grid cannot be coarsened to a level with <= 512 free DOFs: no V-cycle");
  if (g->nlev < 2) return fail(TG_EINVAL, "the adaptive stack needs at least two levels");
  if (restart < 0 || restart > TG_AD_MAX_RESTART || so->inner_steps < 0 || so->inner_steps > TG_AD_MAX_RESTART ||
      so->coarse_steps < 0 || so->coarse_steps > TG_AD_MAX_RESTART)
    return fail(TG_EINVAL, "restart, inner and coarse steps must lie in [0, TG_AD_MAX_RESTART]");
  if (so->nu_pre < 1 || so->nu_pre > ST_MAX_DEGREE || so->nu_post < 1 || so->nu_post > ST_MAX_DEGREE)
    return fail(TG_EINVAL, "Chebyshev degrees must lie in [1, 16]");
  if (so->power_iters < 1 || so->power_iters > 1000) return fail(TG_EINVAL, "power_iters must lie in [1, 1000]");
  if (!(so->lo > 0.0) || !(so->hi > so->lo) || !std::isfinite(so->hi))
    return fail(TG_EINVAL, "need 0 < lo < hi, finite");
  if (!(so->theta >= 0.0) || !std::isfinite(so->theta)) return fail(TG_EINVAL, "theta must be finite and >= 0");
  L.init(g, restart, so->inner_steps, true, so->coarse_steps);
  if (!ws_d) return fail(TG_EINVAL, "NULL workspace");
  if (ws_bytes < L.total) return fail(TG_EWORKSPACE, "stack workspace too small");
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

void tg_default_stack_opts(tg_stack_opts* so) {
  if (!so) return;
  so->inner_steps = 20;
  so->coarse_steps = 10;
  so->nu_pre = 2;
  so->nu_post = 2;
  so->power_iters = 10;
  so->lo = 0.1;
  so->hi = 1.1;
  so->theta = 0.95;
}

int tg_stack_workspace_bytes(const tg_grid* g, int restart, const tg_stack_opts* so, size_t* bytes) {
  if (!g || !so || !bytes) return fail(TG_EINVAL, "NULL argument");
  if (restart < 0 || restart > TG_AD_MAX_RESTART || so->inner_steps < 0 || so->inner_steps > TG_AD_MAX_RESTART ||
      so->coarse_steps < 0 || so->coarse_steps > TG_AD_MAX_RESTART)
    return fail(TG_EINVAL, "restart, inner and coarse steps must lie in [0, TG_AD_MAX_RESTART]");
  Layout L;
  L.init(g, restart, so->inner_steps, true, so->coarse_steps);
  *bytes = L.total;
  return TG_OK;
}

int tg_stack_lambdas(tg_grid* g, const tg_stack_opts* so, void* ws_d, size_t ws_bytes, double* lams_h,
                     void* stream) {
  if (!lams_h) return fail(TG_EINVAL, "NULL argument");
  Layout L;
  int rc = stack_check(g, so, 0, ws_d, ws_bytes, L);
  if (rc) return rc;
  Ctx c{g, (hipStream_t)stream, TG_F64, L, (char*)ws_d, {}};
  c.stack = true;
  c.so = *so;
  if ((rc = batch_set_active(g->self, {0}, c.s))) return rc;
  if ((rc = stack_setup(c))) return rc;
  std::copy(c.lam, c.lam + g->nlev - 1, lams_h);
  return TG_OK;
}

int tg_stack_precondition(tg_grid* g, const double* v_d, double* z_d, const tg_stack_opts* so,
                          const double* lams_h, void* ws_d, size_t ws_bytes, tg_stack_log* log_h, void* stream) {
  if (!v_d || !z_d) return fail(TG_EINVAL, "NULL vector");
  Layout L;
  int rc = stack_check(g, so, 0, ws_d, ws_bytes, L);
  if (rc) return rc;
  Ctx c{g, (hipStream_t)stream, TG_F64, L, (char*)ws_d, {}};
  c.stack = true;
  c.so = *so;
  if ((rc = batch_set_active(g->self, {0}, c.s))) return rc;
  if (lams_h) {
    for (int l = 0; l < g->nlev - 1; ++l)
      if (!(lams_h[l] > 0.0) || !std::isfinite(lams_h[l])) return fail(TG_EINVAL, "lambda estimates must be > 0");
    std::copy(lams_h, lams_h + g->nlev - 1, c.lam);
  } else if ((rc = stack_setup(c))) {
    return rc;
  }
  if ((rc = stack_apply(c, v_d, z_d))) return rc;
  double lg[3] = {0.0, 0.0, 0.0}, acc = 0.0;
  TG_HIP(hipMemcpyAsync(lg, c.stk(), sizeof(lg), hipMemcpyDeviceToHost, c.s));
  TG_HIP(hipMemcpyAsync(&acc, c.isc() + IS_ACC, sizeof(double), hipMemcpyDeviceToHost, c.s));
  TG_HIP(hipStreamSynchronize(c.s));
  if (log_h) *log_h = {lg[ST_ALPHA], lg[ST_RATIO], lg[ST_OK] != 0.0 ? 1 : 0, acc != 0.0 ? 1 : 0};
  return TG_OK;
}

int tg_stack_solve(tg_grid* g, const double* f_d, double* u_d, const tg_solver_opts* o, const tg_stack_opts* so,
                   void* ws_d, size_t ws_bytes, tg_solve_result* res, double* hist_h, tg_stack_log* log_h,
                   int* n_applied_h, double* lams_h, void* stream) {
  if (!f_d || !u_d || !o || !res) return fail(TG_EINVAL, "NULL argument");
  if (o->restart < 1) return fail(TG_EINVAL, "restart must be >= 1");
  if (o->max_iters < 0 || !(o->tol >= 0.0)) return fail(TG_EINVAL, "need max_iters >= 0 and tol >= 0");
  if (o->cgs_passes < 1 || o->cgs_passes > 3) return fail(TG_EINVAL, "cgs_passes must be 1, 2 or 3");
  Layout L;
  int rc = stack_check(g, so, o->restart, ws_d, ws_bytes, L);
  if (rc) return rc;
  Ctx c{g, (hipStream_t)stream, TG_F64, L, (char*)ws_d, {}};
  c.stack = true;
  c.so = *so;
  if ((rc = batch_set_active(g->self, {0}, c.s))) return rc;
  if ((rc = stack_setup(c))) return rc;
  Krylov outer{c.vec(L.oV, 0), c.vec(L.oZ, 0), L.m};
  Outcome out;
  auto M = [&c](const double* v, double* z) { return stack_apply(c, v, z); };
  if ((rc = fgmres(c, outer, f_d, u_d, o->max_iters, o->tol, o->cgs_passes == 1 ? 1 : 2, o->breakdown, M, out)))
    return rc;
  TG_HIP(hipStreamSynchronize(c.s));
  res->iterations = out.iters;
  res->outcome = out.outcome;
  res->proj_eta = out.hist.back();
  res->true_eta = -1.0;
  if (hist_h) std::memcpy(hist_h, out.hist.data(), sizeof(double) * out.hist.size());
  const int na = (int)std::min<size_t>(c.slog.size(), (size_t)o->max_iters + 1);
  if (log_h) std::copy(c.slog.begin(), c.slog.begin() + na, log_h);
  if (n_applied_h) *n_applied_h = (int)c.slog.size();
  if (lams_h) std::copy(c.lam, c.lam + g->nlev - 1, lams_h);
  return TG_OK;
}

int tg_stack_select_floor(tg_grid* g, const double* rho_d, const double* f_d, const tg_policy* pol,
                          const tg_stack_opts* so, void* ws_d, size_t ws_bytes, double* u_d,
                          tg_policy_result* out, void* stream) {
  if (!g || !rho_d || !f_d || !pol || !so || !u_d || !out) return fail(TG_EINVAL, "NULL argument");
  if (pol->n_rungs < 1 || pol->n_rungs > TG_MAX_RUNGS) return fail(TG_EINVAL, "bad policy rungs");
  for (int r = 0; r < pol->n_rungs; ++r)
    if (!(pol->rungs[r] > 0 && pol->rungs[r] <= 1)) return fail(TG_EINVAL, "rungs must be in (0, 1]");
  if (pol->probe_iters < 0 || pol->probe_restart < 1) return fail(TG_EINVAL, "bad probe settings");
  hipStream_t s = (hipStream_t)stream;
  std::memset(out, 0, sizeof(*out));
  int rc;
  // ---- probe at the original floor (its iterate is never returned)
  if ((rc = tg_set_density(g, rho_d, pol->p, pol->rungs[0], stream))) return rc;
  tg_solver_opts po = pol->solve;
  po.restart = pol->probe_restart;
  po.max_iters = pol->probe_iters;
  std::vector<double> h((size_t)std::max(po.max_iters, std::max(pol->solve.max_iters, 0)) + 1);
  tg_solve_result res{};
  if ((rc = tg_stack_solve(g, f_d, u_d, &po, so, ws_d, ws_bytes, &res, h.data(), nullptr, nullptr, nullptr,
                           stream)))
    return rc;
  probe_feats(h.data(), res.iterations, &out->r50, &out->r100);
  out->probe_iters = res.iterations;
  out->iters_probe = res.iterations;
  // ---- first rung: Eq. trigger, the network or a fixed rung
  int k0 = rule_fires(pol, out->r50, out->r100) ? std::min(1, pol->n_rungs - 1) : 0;
  std::vector<std::array<float, 8>> feats(1);
  feats[0].fill(0.f);
  feats[0][0] = (float)std::log10(std::max(out->r50, 1e-300));
  feats[0][1] = (float)std::log10(std::max(out->r100, 1e-300));
  const bool use_mlp = pol->selector == TG_SELECT_MLP && pol->mlp;
  if (use_mlp || pol->want_features)
    if ((rc = density_features(g->self, {0}, &rho_d, pol->p, pol->rungs[0], feats, s))) return rc;
  if (use_mlp) {
    std::vector<int> pred;
    if ((rc = mlp_select(pol->mlp, feats, pred, s))) return rc;
    k0 = std::min(std::max(pred[0], 0), pol->n_rungs - 1);
  } else if (pol->selector == TG_SELECT_FIXED) {
    k0 = std::min(std::max(pol->fixed_rung, 0), pol->n_rungs - 1);
  }
  out->k0 = k0;
  out->rung = -1;
  out->floor = -1.0;
  for (int q = 0; q < 8; ++q) out->features[q] = feats[0][q];
  // ---- guarded ladder: independent solve per rung, recomputed FP64 residual
  for (int r = k0; r < pol->n_rungs && out->rung < 0; ++r) {
    if ((rc = tg_set_density(g, rho_d, pol->p, pol->rungs[r], stream))) return rc;
    if ((rc = tg_stack_solve(g, f_d, u_d, &pol->solve, so, ws_d, ws_bytes, &res, nullptr, nullptr, nullptr,
                             nullptr, stream)))
      return rc;
    double eta = 0.0;
    if ((rc = tg_true_residual(g, f_d, u_d, &eta, stream))) return rc;
    auto& A = out->attempts[out->n_attempts++];
    A.rung = r;
    A.floor = pol->rungs[r];
    A.iterations = res.iterations;
    A.outcome = res.outcome;
    A.proj_eta = res.proj_eta;
    A.true_eta = eta;
    A.accepted = (eta <= pol->tau) && std::isfinite(eta);
    if (A.accepted) {
      out->rung = r;
      out->floor = A.floor;
      out->iters_selected = A.iterations;
    } else {
      out->iters_rejected += A.iterations;
    }
  }
  if (out->rung < 0) {
    const size_t n_dof = 3ull * (g->nx + 1) * (g->ny + 1) * (g->nz + 1);
    TG_HIP(hipMemsetAsync(u_d, 0, n_dof * sizeof(double), s));
  }
  TG_HIP(hipStreamSynchronize(s));
  return TG_OK;
}

}  // extern "C"
