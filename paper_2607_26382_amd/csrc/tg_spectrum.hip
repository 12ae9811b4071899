// Extreme eigenvalues of the frozen free-DOF operator K(rho_min) (Eq.
// frozen_operator) and so its condition number, the quantity behind the
// conditioning indicator kappa * eps and the floor screen of Sec. 4.2
// (Eq. screen).
//
// lambda_max: Lanczos on K (three-term recurrence, no reorthogonalization:
// the largest Ritz value converges long before orthogonality loss matters),
// the tridiagonal's largest eigenvalue by Sturm bisection on the host.
// lambda_min: single-vector LOBPCG (Knyazev 2001) preconditioned by one
// V-cycle of the library's multigrid: Rayleigh-Ritz on [x, w, p] each step,
// all Gram entries from one fused pass over the six vectors x, w, p, Kx, Kw,
// Kp, the 3 x 3 generalized eigenproblem on the host.  Apply, V-cycle and
// vector passes are the library's kernels; sums run in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "tg_internal.h"

namespace tg {
namespace {

constexpr int SP_BLOCK = 256;
constexpr int SP_NVEC = 6;       // x, w, p, Kx, Kw, Kp
constexpr int SP_NDOT = 12;      // the Gram entries

struct VecSet {
  const double* v[SP_NVEC];
};
struct Pairs {
  unsigned char a[SP_NDOT], b[SP_NDOT];
  int n;
};
struct Comb {
  double c[4][SP_NVEC];   // out[o] = sum_j c[o][j] in[j]
  double* out[4];
  const double* in[SP_NVEC];
  int n_out;
};

int nblk(long long n) { return (int)std::max<long long>(1, std::min<long long>(1024, (n + SP_BLOCK - 1) / SP_BLOCK)); }

// Counter-based start vector on the free DOFs: a multiplicative hash of the
// DOF index mapped to [-0.5, 0.5) (deterministic; any vector with components
// along the extreme eigenvectors serves).
__global__ __launch_bounds__(SP_BLOCK) void k_sp_start(double* __restrict__ x, long long n, int NX) {
  for (long long d = (long long)blockIdx.x * SP_BLOCK + threadIdx.x; d < n; d += (long long)gridDim.x * SP_BLOCK) {
    const long long node = d / 3;
    const unsigned h = (unsigned)((unsigned long long)(d + 1) * 2654435761ull) ^ 0x9e3779b9u;
    const unsigned g = h * 0x85ebca6bu;
    x[d] = (node % NX == 0) ? 0.0 : (double)(g >> 8) * (1.0 / 16777216.0) - 0.5;
  }
}

// part[block][q] = sum_i v[a_q][i] v[b_q][i]
__global__ __launch_bounds__(SP_BLOCK) void k_sp_dots(VecSet V, Pairs P, long long n, double* __restrict__ part) {
  __shared__ double red[SP_BLOCK / 64][SP_NDOT];
  double acc[SP_NDOT];
#pragma unroll
  for (int q = 0; q < SP_NDOT; ++q) acc[q] = 0.0;
  for (long long i = (long long)blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * SP_BLOCK) {
#pragma unroll
    for (int q = 0; q < SP_NDOT; ++q)
      if (q < P.n) acc[q] += V.v[P.a[q]][i] * V.v[P.b[q]][i];
  }
#pragma unroll
  for (int q = 0; q < SP_NDOT; ++q) {
    double s = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < SP_NDOT && (int)threadIdx.x < P.n) {
    double s = 0.0;
    for (int w = 0; w < SP_BLOCK / 64; ++w) s += red[w][threadIdx.x];
    part[(long long)blockIdx.x * SP_NDOT + threadIdx.x] = s;
  }
}

// Linear combinations; every output element is formed from the inputs'
// values at that index before any output is written (outputs may alias).
__global__ __launch_bounds__(SP_BLOCK) void k_sp_comb(Comb C, long long n) {
  for (long long i = (long long)blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * SP_BLOCK) {
    double in[SP_NVEC];
#pragma unroll
    for (int j = 0; j < SP_NVEC; ++j) in[j] = C.in[j] ? C.in[j][i] : 0.0;
    double o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < SP_NVEC; ++j) s += C.c[k][j] * in[j];
      o[k] = s;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < C.n_out) C.out[k][i] = o[k];
  }
}

__global__ __launch_bounds__(SP_BLOCK) void k_sp_to32(const double* __restrict__ a, float* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * SP_BLOCK)
    b[i] = (float)a[i];
}
__global__ __launch_bounds__(SP_BLOCK) void k_sp_to64(const float* __restrict__ a, double* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * SP_BLOCK)
    b[i] = (double)a[i];
}

struct Ctx {
  tg_grid* g;
  hipStream_t s;
  long long n;
  double* part;
  int cap;          // partial-sum capacity in doubles
};

int dots(Ctx& c, const VecSet& V, const Pairs& P, double* out) {
  const int nb = nblk(c.n);
  if ((long long)nb * SP_NDOT > c.cap) return fail(TG_EINVAL, "partial buffer too small");
  k_sp_dots<<<nb, SP_BLOCK, 0, c.s>>>(V, P, c.n, c.part);
  TG_HIP(hipGetLastError());
  std::vector<double> h((size_t)nb * SP_NDOT);
  TG_HIP(hipMemcpyAsync(h.data(), c.part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c.s));
  TG_HIP(hipStreamSynchronize(c.s));
  for (int q = 0; q < P.n; ++q) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += h[(size_t)b * SP_NDOT + q];
    out[q] = s;
  }
  return TG_OK;
}

int comb(Ctx& c, const Comb& C) {
  k_sp_comb<<<nblk(c.n), SP_BLOCK, 0, c.s>>>(C, c.n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int applyK(Ctx& c, const double* x, double* y) { return tg_apply_K(c.g, x, y, TG_F64, c.s); }

// z = M^-1 r, one V-cycle at precision prec (FP32 forms through float copies)
int precond(Ctx& c, int prec, const double* r, double* z, float* r32, float* z32) {
  if (prec == TG_F64) return tg_vcycle(c.g, r, z, TG_F64, c.s);
  k_sp_to32<<<nblk(c.n), SP_BLOCK, 0, c.s>>>(r, r32, c.n);
  TG_HIP(hipGetLastError());
  const int rc = tg_vcycle(c.g, r32, z32, prec, c.s);
  if (rc) return rc;
  k_sp_to64<<<nblk(c.n), SP_BLOCK, 0, c.s>>>(z32, z, c.n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

// number of eigenvalues of the symmetric tridiagonal (a, b) below x
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double bb = i ? b[i - 1] * b[i - 1] : 0.0;
    q = a[i] - x - (i ? bb / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}

double tridiag_max(const std::vector<double>& a, const std::vector<double>& b) {
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < a.size(); ++i) {
    const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  const int n = (int)a.size();
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(hi), std::fabs(lo)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(a, b, mid) < n) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Smallest eigenpair of A c = mu B c (m <= 3, B symmetric positive
// definite): Cholesky B = L L^T, Jacobi sweeps on L^-1 A L^-T.  Returns false
// if B is not numerically positive definite.
bool small_geneig(int m, const double A[3][3], const double B[3][3], double& mu, double c[3]) {
  double L[3][3] = {};
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = B[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(s > 1e-12 * B[i][i])) return false;
        L[i][i] = std::sqrt(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  // Li = L^-1
  double Li[3][3] = {};
  for (int i = 0; i < m; ++i) {
    Li[i][i] = 1.0 / L[i][i];
    for (int j = 0; j < i; ++j) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[i][k] * Li[k][j];
      Li[i][j] = -s / L[i][i];
    }
  }
  double C[3][3] = {}, V[3][3] = {};
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k)
        for (int l = 0; l < m; ++l) s += Li[i][k] * A[k][l] * Li[j][l];
      C[i][j] = s;
    }
  for (int i = 0; i < m; ++i) V[i][i] = 1.0;
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) off += C[i][j] * C[i][j];
    if (off < 1e-30 * (C[0][0] * C[0][0] + 1e-300)) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        if (C[p][q] == 0.0) continue;
        const double th = 0.5 * (C[q][q] - C[p][p]) / C[p][q];
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < m; ++k) {   // columns p, q
          const double a = C[k][p], b = C[k][q];
          C[k][p] = cs * a - sn * b;
          C[k][q] = sn * a + cs * b;
        }
        for (int k = 0; k < m; ++k) {   // rows p, q
          const double a = C[p][k], b = C[q][k];
          C[p][k] = cs * a - sn * b;
          C[q][k] = sn * a + cs * b;
        }
        for (int k = 0; k < m; ++k) {
          const double a = V[k][p], b = V[k][q];
          V[k][p] = cs * a - sn * b;
          V[k][q] = sn * a + cs * b;
        }
      }
  }
  int im = 0;
  for (int i = 1; i < m; ++i)
    if (C[i][i] < C[im][im]) im = i;
  mu = C[im][im];
  // c = L^-T y, y = column im of V
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += Li[k][i] * V[k][im];
    c[i] = s;
  }
  for (int i = m; i < 3; ++i) c[i] = 0.0;
  return true;
}

}  // namespace
}  // namespace tg

using namespace tg;

extern "C" {

int tg_spectrum_workspace_bytes(const tg_grid* g, size_t* bytes) {
  if (!g || !bytes) return fail(TG_EINVAL, "NULL argument");
  const size_t nd = (size_t)g->lv[0].n_dof;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  *bytes = 7 * al(nd * sizeof(double)) + 2 * al(nd * sizeof(float));
  return TG_OK;
}

int tg_extreme_eigenvalues(tg_grid* g, int prec, int max_iters, double tol, void* ws_d, size_t ws_bytes,
                           tg_spectrum_result* out, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!g->density_set) return fail(TG_ESTATE, "set_density first");
  if (!ws_d || !out) return fail(TG_EINVAL, "NULL argument");
  if (prec < TG_F64 || prec > TG_BF16X3MFMA) return fail(TG_EINVAL, "bad precision");
  if (max_iters < 2 || !(tol > 0)) return fail(TG_EINVAL, "need max_iters >= 2 and tol > 0");
  size_t need = 0;
  tg_spectrum_workspace_bytes(g, &need);
  if (ws_bytes < need) return fail(TG_EWORKSPACE, "spectrum workspace too small");
  std::memset(out, 0, sizeof(*out));
  Ctx c{g, (hipStream_t)stream, (long long)g->lv[0].n_dof, g->desc.part,
        (int)std::min<long long>(1 << 30, (long long)TG_PART_W * g->lv[0].n_chunks)};
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* w8 = (char*)ws_d;
  double* V[7];
  for (int i = 0; i < 7; ++i, w8 += al((size_t)c.n * sizeof(double))) V[i] = (double*)w8;
  float* r32 = (float*)w8;
  float* z32 = (float*)(w8 + al((size_t)c.n * sizeof(float)));
  double *x = V[0], *w = V[1], *p = V[2], *Kx = V[3], *Kw = V[4], *Kp = V[5], *r = V[6];
  int rc;
  const int NX = g->nx + 1;

  // ---- lambda_max: Lanczos on K from the hashed start vector
  k_sp_start<<<nblk(c.n), SP_BLOCK, 0, c.s>>>(x, c.n, NX);
  TG_HIP(hipGetLastError());
  {
    double d[SP_NDOT];
    Pairs P{};
    P.n = 1;
    P.a[0] = 0; P.b[0] = 0;
    VecSet VS{{x, w, p, Kx, Kw, Kp}};
    if ((rc = dots(c, VS, P, d))) return rc;
    Comb C{};
    C.n_out = 1; C.out[0] = x; C.in[0] = x; C.c[0][0] = 1.0 / std::sqrt(d[0]);
    if ((rc = comb(c, C))) return rc;
    // v_prev = p (zero), v = x, w = K v - beta v_prev
    std::vector<double> A, Bt;
    double beta = 0.0, prev = 0.0, theta = 0.0;
    double *vp = p, *v = x, *wk = w;
    TG_HIP(hipMemsetAsync(vp, 0, sizeof(double) * c.n, c.s));
    for (int j = 0; j < max_iters; ++j) {
      if ((rc = applyK(c, v, wk))) return rc;
      VecSet S{{v, wk, vp, Kx, Kw, Kp}};
      Pairs Q{};
      Q.n = 1; Q.a[0] = 0; Q.b[0] = 1;
      double alpha;
      if ((rc = dots(c, S, Q, &alpha))) return rc;
      Comb U{};
      U.n_out = 1; U.out[0] = wk; U.in[0] = wk; U.in[1] = v; U.in[2] = vp;
      U.c[0][0] = 1.0; U.c[0][1] = -alpha; U.c[0][2] = -beta;
      if ((rc = comb(c, U))) return rc;
      Q.a[0] = 1; Q.b[0] = 1;
      double nn;
      if ((rc = dots(c, S, Q, &nn))) return rc;
      A.push_back(alpha);
      beta = std::sqrt(std::max(nn, 0.0));
      theta = tridiag_max(A, Bt);
      out->iters_max = j + 1;
      if (j >= 4 && std::fabs(theta - prev) <= 1e-12 * theta) break;
      prev = theta;
      if (!(beta > 1e-300)) break;
      Bt.push_back(beta);
      // v_prev <- v, v <- w / beta, w <- (old v_prev storage)
      Comb N{};
      N.n_out = 1; N.out[0] = wk; N.in[0] = wk; N.c[0][0] = 1.0 / beta;
      if ((rc = comb(c, N))) return rc;
      double* t = vp;
      vp = v;
      v = wk;
      wk = t;
    }
    out->lambda_max = theta;
  }

  // ---- lambda_min: LOBPCG preconditioned by the V-cycle
  k_sp_start<<<nblk(c.n), SP_BLOCK, 0, c.s>>>(x, c.n, NX);
  TG_HIP(hipGetLastError());
  if ((rc = applyK(c, x, Kx))) return rc;
  double lam = 0.0, res = 0.0;
  bool have_p = false;
  {
    VecSet VS{{x, w, p, Kx, Kw, Kp}};
    Pairs P{};
    P.n = 2;
    P.a[0] = 0; P.b[0] = 0;    // x.x
    P.a[1] = 0; P.b[1] = 3;    // x.Kx
    double d[SP_NDOT];
    if ((rc = dots(c, VS, P, d))) return rc;
    const double s = 1.0 / std::sqrt(d[0]);
    Comb C{};
    C.n_out = 2; C.out[0] = x; C.out[1] = Kx; C.in[0] = x; C.in[3] = Kx;
    C.c[0][0] = s; C.c[1][3] = s;
    if ((rc = comb(c, C))) return rc;
    lam = d[1] / d[0];
  }
  for (int it = 0; it < max_iters; ++it) {
    // r = Kx - lam x
    Comb R{};
    R.n_out = 1; R.out[0] = r; R.in[0] = x; R.in[3] = Kx; R.c[0][0] = -lam; R.c[0][3] = 1.0;
    if ((rc = comb(c, R))) return rc;
    {
      VecSet VS{{x, r, p, Kx, Kw, Kp}};
      Pairs P{};
      P.n = 2; P.a[0] = 1; P.b[0] = 1; P.a[1] = 3; P.b[1] = 3;
      double d[SP_NDOT];
      if ((rc = dots(c, VS, P, d))) return rc;
      res = std::sqrt(std::max(d[0], 0.0)) / std::sqrt(d[1]);   // ||Kx - lam x|| / ||Kx||
    }
    out->iters_min = it;
    if (res <= tol) {
      out->converged = 1;
      break;
    }
    if ((rc = precond(c, prec, r, w, r32, z32))) return rc;
    if ((rc = applyK(c, w, Kw))) return rc;
    VecSet VS{{x, w, p, Kx, Kw, Kp}};
    // Gram entries: B = S^T S and A = S^T K S over S = [x, w, p]
    Pairs P{};
    const unsigned char pa[SP_NDOT] = {0, 0, 0, 1, 1, 2, 0, 0, 0, 1, 1, 2};
    const unsigned char pb[SP_NDOT] = {0, 1, 2, 1, 2, 2, 3, 4, 5, 4, 5, 5};
    for (int q = 0; q < SP_NDOT; ++q) { P.a[q] = pa[q]; P.b[q] = pb[q]; }
    P.n = SP_NDOT;
    double d[SP_NDOT];
    if ((rc = dots(c, VS, P, d))) return rc;
    const double Bm[3][3] = {{d[0], d[1], d[2]}, {d[1], d[3], d[4]}, {d[2], d[4], d[5]}};
    const double Am[3][3] = {{d[6], d[7], d[8]}, {d[7], d[9], d[10]}, {d[8], d[10], d[11]}};
    // scale w and p to unit length in the small problem
    double sc[3] = {1.0, 1.0 / std::sqrt(std::max(Bm[1][1], 1e-300)), have_p ? 1.0 / std::sqrt(std::max(Bm[2][2], 1e-300)) : 0.0};
    int m = have_p ? 3 : 2;
    double As[3][3], Bs[3][3], cvec[3], mu;
    bool ok = false;
    while (!ok && m >= 2) {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          As[i][j] = Am[i][j] * sc[i] * sc[j];
          Bs[i][j] = Bm[i][j] * sc[i] * sc[j];
        }
      ok = small_geneig(m, As, Bs, mu, cvec);
      if (!ok) --m;     // drop p (then w) when the basis has degenerated
    }
    if (!ok) break;
    for (int i = 0; i < 3; ++i) cvec[i] *= (i < m ? sc[i] : 0.0);
    // x <- c0 x + c1 w + c2 p, p <- c1 w + c2 p, and the same for K*
    Comb U{};
    U.n_out = 4;
    U.out[0] = x; U.out[1] = p; U.out[2] = Kx; U.out[3] = Kp;
    U.in[0] = x; U.in[1] = w; U.in[2] = have_p ? p : nullptr;
    U.in[3] = Kx; U.in[4] = Kw; U.in[5] = have_p ? Kp : nullptr;
    U.c[0][0] = cvec[0]; U.c[0][1] = cvec[1]; U.c[0][2] = cvec[2];
    U.c[1][1] = cvec[1]; U.c[1][2] = cvec[2];
    U.c[2][3] = cvec[0]; U.c[2][4] = cvec[1]; U.c[2][5] = cvec[2];
    U.c[3][4] = cvec[1]; U.c[3][5] = cvec[2];
    if ((rc = comb(c, U))) return rc;
    have_p = true;
    // renormalize x (and Kx) and p (and Kp)
    {
      VecSet S2{{x, w, p, Kx, Kw, Kp}};
      Pairs Q{};
      Q.n = 3; Q.a[0] = 0; Q.b[0] = 0; Q.a[1] = 2; Q.b[1] = 2; Q.a[2] = 0; Q.b[2] = 3;
      double e[SP_NDOT];
      if ((rc = dots(c, S2, Q, e))) return rc;
      const double sx = 1.0 / std::sqrt(e[0]), sp = e[1] > 0 ? 1.0 / std::sqrt(e[1]) : 0.0;
      Comb Nm{};
      Nm.n_out = 4;
      Nm.out[0] = x; Nm.out[1] = p; Nm.out[2] = Kx; Nm.out[3] = Kp;
      Nm.in[0] = x; Nm.in[2] = p; Nm.in[3] = Kx; Nm.in[5] = Kp;
      Nm.c[0][0] = sx; Nm.c[1][2] = sp; Nm.c[2][3] = sx; Nm.c[3][5] = sp;
      if ((rc = comb(c, Nm))) return rc;
      lam = e[2] / e[0];
    }
    out->iters_min = it + 1;
  }
  out->lambda_min = lam;
  out->resid_min = res;
  out->kappa = out->lambda_max / lam;
  return TG_OK;
}

}  // extern "C"
