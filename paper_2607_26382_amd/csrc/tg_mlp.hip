// Learned first-floor selector: an 8-64-64-4 network with exact-erf GELU,
// softmax cross-entropy and Adam, trained and evaluated by the kernels below,
// and the six density statistics it reads besides the two probe features.
//
// Network kernels work one wavefront per sample: lane j owns hidden unit j of
// both hidden layers, cross-lane vectors move by __shfl, W2 sits in LDS (padded
// rows, so both its rows and its columns read without bank conflicts).  Every
// sum runs in a fixed order and the gradient is reduced over a fixed set of
// per-wave partials, so training is bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "tg_internal.h"

namespace {
constexpr int NIN = 8, NH = 64, NOUT = 4;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NOUT * NH, NPARAM = OFF_B3 + NOUT;
static_assert(NPARAM == 4996, "parameter count");
constexpr int GSTRIDE = 5120;     // padded stride of one per-wave gradient partial
constexpr int MAX_WAVES = 256;    // waves (partials) of one gradient pass
constexpr int FWD_MAX_BLOCKS = 1024;
}  // namespace

struct tg_mlp {
  float* P = nullptr;      // parameters (NPARAM)
  float* M = nullptr;      // Adam first moments
  float* V = nullptr;      // Adam second moments
  float* G = nullptr;      // last reduced gradient
  float* part = nullptr;   // MAX_WAVES x GSTRIDE gradient partials
  float* lpart = nullptr;  // MAX_WAVES loss partials
  float* loss = nullptr;   // 1
  float* mean = nullptr;   // 8 standardization offsets
  float* sd = nullptr;     // 8 standardization scales
  float* x = nullptr;      // max_batch x 8 staging (selector calls)
  float* logits = nullptr; // max_batch x 4
  int* pred = nullptr;     // max_batch
  int max_batch = 0;
  long long t = 0;         // Adam steps taken
  bool params_set = false;
};

namespace tg {
namespace {

__device__ __forceinline__ float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
// d/da GELU(a) = Phi(a) + a phi(a)
__device__ __forceinline__ float gelu_d(float a) {
  const float Phi = 0.5f * (1.0f + erff(a * 0.70710678118654752f));
  const float phi = 0.39894228040143268f * expf(-0.5f * a * a);
  return Phi + a * phi;
}
__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;   // identical in every lane: each butterfly stage adds commuted pairs
}

struct Fwd {
  float xs[NIN];
  float a1, h1, a2, h2;
  float lg[NOUT];
};

// Forward pass of one sample by one wavefront (lane = hidden unit).
__device__ __forceinline__ void fwd_sample(const float* __restrict__ x, const float* mu, const float* sd,
                                           const float* w1, float b1, const float (*sW2)[NH + 1], float b2,
                                           const float* w3, const float* b3, int lane, Fwd& f) {
#pragma unroll
  for (int k = 0; k < NIN; ++k) f.xs[k] = (x[k] - mu[k]) / sd[k];
  float a = 0.f;
#pragma unroll
  for (int k = 0; k < NIN; ++k) a = fmaf(w1[k], f.xs[k], a);
  f.a1 = a + b1;
  f.h1 = gelu(f.a1);
  a = 0.f;
#pragma unroll 8
  for (int k = 0; k < NH; ++k) a = fmaf(sW2[lane][k], __shfl(f.h1, k, 64), a);
  f.a2 = a + b2;
  f.h2 = gelu(f.a2);
#pragma unroll
  for (int c = 0; c < NOUT; ++c) f.lg[c] = wave_sum_f(w3[c] * f.h2) + b3[c];
}

__device__ __forceinline__ void load_lane_params(const float* __restrict__ P, int lane, float* w1, float& b1,
                                                 float& b2, float* w3, float* b3) {
#pragma unroll
  for (int k = 0; k < NIN; ++k) w1[k] = P[OFF_W1 + lane * NIN + k];
  b1 = P[OFF_B1 + lane];
  b2 = P[OFF_B2 + lane];
#pragma unroll
  for (int c = 0; c < NOUT; ++c) {
    w3[c] = P[OFF_W3 + c * NH + lane];
    b3[c] = P[OFF_B3 + c];
  }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P, const float* __restrict__ mean,
                                                     const float* __restrict__ sdv, const float* __restrict__ x,
                                                     int B, float* __restrict__ logits, int* __restrict__ pred) {
  __shared__ float sW2[NH][NH + 1];
  for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) sW2[i / NH][i % NH] = P[OFF_W2 + i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float w1[NIN], b1, b2, w3[NOUT], b3[NOUT], mu[NIN], sd[NIN];
  load_lane_params(P, lane, w1, b1, b2, w3, b3);
#pragma unroll
  for (int k = 0; k < NIN; ++k) {
    mu[k] = mean[k];
    sd[k] = sdv[k];
  }
  const int nw = gridDim.x * 4;
  for (int s = blockIdx.x * 4 + wv; s < B; s += nw) {
    Fwd f;
    fwd_sample(x + (long long)s * NIN, mu, sd, w1, b1, sW2, b2, w3, b3, lane, f);
    if (lane == 0) {
      int best = 0;
      float bv = f.lg[0];
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {
        logits[(long long)s * NOUT + c] = f.lg[c];
        if (f.lg[c] > bv) {   // strict: ties go to the lower rung
          bv = f.lg[c];
          best = c;
        }
      }
      if (pred) pred[s] = best;
    }
  }
}

// Per-wave gradient partials of the mean cross-entropy (and the summed
// per-sample loss).  Wave w handles samples w, w + nw, ...; every one of the
// gridDim.x * 4 waves writes its partial, zero if it had no sample.
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ P, const float* __restrict__ mean,
                                                  const float* __restrict__ sdv, const float* __restrict__ x,
                                                  const int* __restrict__ y, int B, float invB,
                                                  float* __restrict__ part, float* __restrict__ lpart) {
  __shared__ float sW2[NH][NH + 1];
  for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) sW2[i / NH][i % NH] = P[OFF_W2 + i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gw = blockIdx.x * 4 + wv, nw = gridDim.x * 4;
  float w1[NIN], b1, b2, w3[NOUT], b3[NOUT], mu[NIN], sd[NIN];
  load_lane_params(P, lane, w1, b1, b2, w3, b3);
#pragma unroll
  for (int k = 0; k < NIN; ++k) {
    mu[k] = mean[k];
    sd[k] = sdv[k];
  }
  float gW1[NIN] = {}, gW2[NH] = {}, gW3[NOUT] = {}, gb3[NOUT] = {};
  float gb1 = 0.f, gb2 = 0.f, lsum = 0.f;
  for (int s = gw; s < B; s += nw) {
    Fwd f;
    fwd_sample(x + (long long)s * NIN, mu, sd, w1, b1, sW2, b2, w3, b3, lane, f);
    const int ys = y[s];
    float m = f.lg[0];
#pragma unroll
    for (int c = 1; c < NOUT; ++c) m = fmaxf(m, f.lg[c]);
    float e[NOUT], se = 0.f;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      e[c] = expf(f.lg[c] - m);
      se += e[c];
    }
    float lgy = f.lg[0];
#pragma unroll
    for (int c = 1; c < NOUT; ++c) lgy = (c == ys) ? f.lg[c] : lgy;
    lsum += (m + logf(se)) - lgy;      // -log softmax(y) in log-sum-exp form
    float dl[NOUT], dh2 = 0.f;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      dl[c] = (e[c] / se - (c == ys ? 1.f : 0.f)) * invB;
      gW3[c] = fmaf(dl[c], f.h2, gW3[c]);
      gb3[c] += dl[c];
      dh2 = fmaf(w3[c], dl[c], dh2);
    }
    const float dz2 = dh2 * gelu_d(f.a2);
    gb2 += dz2;
#pragma unroll
    for (int k = 0; k < NH; ++k) gW2[k] = fmaf(dz2, __shfl(f.h1, k, 64), gW2[k]);   // register row
    float dh1 = 0.f;
#pragma unroll 8
    for (int i = 0; i < NH; ++i) dh1 = fmaf(sW2[i][lane], __shfl(dz2, i, 64), dh1);
    const float dz1 = dh1 * gelu_d(f.a1);
    gb1 += dz1;
#pragma unroll
    for (int k = 0; k < NIN; ++k) gW1[k] = fmaf(dz1, f.xs[k], gW1[k]);
  }
  float* out = part + (long long)gw * GSTRIDE;
#pragma unroll
  for (int k = 0; k < NIN; ++k) out[OFF_W1 + lane * NIN + k] = gW1[k];
  out[OFF_B1 + lane] = gb1;
#pragma unroll
  for (int k = 0; k < NH; ++k) out[OFF_W2 + lane * NH + k] = gW2[k];
  out[OFF_B2 + lane] = gb2;
#pragma unroll
  for (int c = 0; c < NOUT; ++c) out[OFF_W3 + c * NH + lane] = gW3[c];
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NOUT; ++c) out[OFF_B3 + c] = gb3[c];
    lpart[gw] = lsum;
  }
}

// Sums the nw partials in wave order, stores the gradient and takes one Adam
// step (c1, c2: bias corrections 1/(1 - beta^t)).  Thread NPARAM sums the loss.
__global__ __launch_bounds__(256) void k_mlp_adam(const float* __restrict__ part, const float* __restrict__ lpart,
                                                  int nw, float invB, float lr, float b1, float b2, float eps,
                                                  float c1, float c2, int update, float* __restrict__ P,
                                                  float* __restrict__ M, float* __restrict__ V,
                                                  float* __restrict__ G, float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == NPARAM) {
    float l = 0.f;
    for (int w = 0; w < nw; ++w) l += lpart[w];
    loss[0] = l * invB;
    return;
  }
  if (i > NPARAM) return;
  float g = 0.f;
  for (int w = 0; w < nw; ++w) g += part[(long long)w * GSTRIDE + i];
  G[i] = g;
  if (!update) return;
  const float m = b1 * M[i] + (1.f - b1) * g;
  const float v = b2 * V[i] + (1.f - b2) * g * g;
  M[i] = m;
  V[i] = v;
  P[i] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// ---------------------------------------------------------------------------
// density statistics
__device__ __forceinline__ int ld_lab(const int* lab, long long i) {
  return __hip_atomic_load(lab + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x.  Parents are always smaller than their children, so the walk ends
// within x steps; halving stores point x at an ancestor, which stays valid
// under concurrent merges (trees only ever join).
__device__ int uf_find(int* lab, int x) {
  while (true) {
    const int p = ld_lab(lab, x);
    if (p == x) return x;
    const int q = ld_lab(lab, p);
    if (q == p) return p;
    __hip_atomic_store(lab + x, q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = q;
  }
}

// Joins the trees of a and b by hooking the larger root under the smaller one.
__device__ bool uf_unite(int* lab, int a, int b) {
  for (int it = 0; it < (1 << 20); ++it) {
    a = uf_find(lab, a);
    b = uf_find(lab, b);
    if (a == b) return true;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(lab + a, a, b) == a) return true;
  }
  return false;
}

__device__ __forceinline__ bool solid(const double* rho, long long e) { return rho[e] >= 0.5; }

__global__ __launch_bounds__(256) void k_cc_init(const ProbDesc* __restrict__ probs, const int2* __restrict__ work) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& L = P.lv[0];
  const long long n_e = (long long)L.ex * L.ey * L.ez;
  const long long e = (long long)wi.y * 256 + threadIdx.x;
  if (e >= n_e) return;
  P.cc[e] = solid(P.ext0, e) ? (int)e : -1;
  P.cc[n_e + e] = 0;
}

__global__ __launch_bounds__(256) void k_cc_hook(const ProbDesc* __restrict__ probs, const int2* __restrict__ work,
                                                 int* __restrict__ err) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& L = P.lv[0];
  const long long n_e = (long long)L.ex * L.ey * L.ez;
  const long long e = (long long)wi.y * 256 + threadIdx.x;
  if (e >= n_e || !solid(P.ext0, e)) return;
  const int ex = (int)(e % L.ex), ey = (int)((e / L.ex) % L.ey), ez = (int)(e / ((long long)L.ex * L.ey));
  bool ok = true;
  if (ex + 1 < L.ex && solid(P.ext0, e + 1)) ok = uf_unite(P.cc, (int)e, (int)(e + 1)) && ok;
  if (ey + 1 < L.ey && solid(P.ext0, e + L.ex)) ok = uf_unite(P.cc, (int)e, (int)(e + L.ex)) && ok;
  const long long sz = (long long)L.ex * L.ey;
  if (ez + 1 < L.ez && solid(P.ext0, e + sz)) ok = uf_unite(P.cc, (int)e, (int)(e + sz)) && ok;
  if (!ok) atomicOr(err + wi.x, 4);
}

// After hooking: every element points straight at its root.  The walk does
// not compress, so the only store to lab[e] is this thread's root (a
// concurrent reader sees either the old parent or the root, both ancestors).
__global__ __launch_bounds__(256) void k_cc_root(const ProbDesc* __restrict__ probs, const int2* __restrict__ work) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& L = P.lv[0];
  const long long n_e = (long long)L.ex * L.ey * L.ez;
  const long long e = (long long)wi.y * 256 + threadIdx.x;
  if (e >= n_e || P.cc[e] < 0) return;
  int x = (int)e;
  for (int p = ld_lab(P.cc, x); p != x; p = ld_lab(P.cc, x)) x = p;
  __hip_atomic_store(P.cc + e, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// flag every component that reaches an element on the clamped face (ex = 0)
__global__ __launch_bounds__(256) void k_cc_mark(const ProbDesc* __restrict__ probs, const int2* __restrict__ work) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& L = P.lv[0];
  const long long n_e = (long long)L.ex * L.ey * L.ez;
  const long long e = (long long)wi.y * 256 + threadIdx.x;
  if (e >= n_e || e % L.ex != 0) return;
  const int r = P.cc[e];
  if (r >= 0) P.cc[n_e + r] = 1;
}

// One workgroup per problem: floor fraction, mean, min nonzero, contrast at
// floor rho0, connectivity proxy, log10 of the DOF count.
__global__ __launch_bounds__(256) void k_dstats(const ProbDesc* __restrict__ probs, const int2* __restrict__ work,
                                                double p, double rho0, double* __restrict__ feat) {
  const int pi = work[blockIdx.x].x;
  const ProbDesc& P = probs[pi];
  const LevelDesc& L = P.lv[0];
  const long long n_e = (long long)L.ex * L.ey * L.ez;
  const double* rho = P.ext0;
  double sum = 0.0, mn = INFINITY, mx = -INFINITY;
  long long zeros = 0;
  for (long long e = threadIdx.x; e < n_e; e += 256) {
    const double r = rho[e];
    sum += r;
    if (r == 0.0) {
      ++zeros;
    } else {
      mn = fmin(mn, r);
      mx = fmax(mx, r);
    }
  }
  __shared__ double ss[256], smn[256], smx[256];
  __shared__ long long sz[256];
  ss[threadIdx.x] = sum;
  smn[threadIdx.x] = mn;
  smx[threadIdx.x] = mx;
  sz[threadIdx.x] = zeros;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (threadIdx.x < o) {
      ss[threadIdx.x] += ss[threadIdx.x + o];
      smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + o]);
      smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + o]);
      sz[threadIdx.x] += sz[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  int hits = 0;
  for (int ey = 0; ey < L.ey; ++ey) {
    const long long e = (long long)(L.ex - 1) + (long long)L.ex * ey;   // ez = 0, ex = nx - 1
    const int r = P.cc[e];
    if (r >= 0 && P.cc[n_e + r]) ++hits;
  }
  const bool any = smx[0] > 0.0;
  double contrast = 0.0;
  if (any) {
    const double Emax = rho0 + (1.0 - rho0) * pow(smx[0], p);
    const double Emin = rho0 + (1.0 - rho0) * pow(smn[0], p);
    contrast = log10(Emax / Emin);
  }
  double* o = feat + 8 * pi;
  o[0] = (double)sz[0] / (double)n_e;
  o[1] = ss[0] / (double)n_e;
  o[2] = any ? smn[0] : 0.0;
  o[3] = contrast;
  o[4] = (double)hits / (double)L.ey;
  o[5] = log10(3.0 * (double)L.NX * (double)L.NY * (double)L.NZ);
  o[6] = o[7] = 0.0;
}

int mlp_check(const tg_mlp* m) {
  if (!m) return fail(TG_EINVAL, "NULL MLP handle");
  if (!m->params_set) return fail(TG_ESTATE, "MLP parameters not set");
  return TG_OK;
}

int fwd_launch(const tg_mlp* m, const float* x, int B, float* logits, int* pred, hipStream_t s) {
  if (B <= 0) return TG_OK;
  const int blocks = std::min((B + 3) / 4, FWD_MAX_BLOCKS);
  k_mlp_forward<<<blocks, 256, 0, s>>>(m->P, m->mean, m->sd, x, B, logits, pred);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

}  // namespace

// Selector use inside the policy: raw features (host) -> first rung per
// problem, argmax with ties to the lower rung.
int mlp_select(const tg_mlp* m, const std::vector<std::array<float, 8>>& feats, std::vector<int>& k0,
               hipStream_t s) {
  int rc = mlp_check(m);
  if (rc) return rc;
  const int n = (int)feats.size();
  k0.assign(n, 0);
  std::vector<float> xh(8 * (size_t)m->max_batch);
  for (int b0 = 0; b0 < n; b0 += m->max_batch) {
    const int B = std::min(m->max_batch, n - b0);
    for (int i = 0; i < B; ++i) std::memcpy(&xh[8 * (size_t)i], feats[b0 + i].data(), 8 * sizeof(float));
    TG_HIP(hipMemcpyAsync(m->x, xh.data(), sizeof(float) * 8 * B, hipMemcpyHostToDevice, s));
    if ((rc = fwd_launch(m, m->x, B, m->logits, m->pred, s))) return rc;
    TG_HIP(hipMemcpyAsync(k0.data() + b0, m->pred, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
  }
  return TG_OK;
}

// Six density statistics per problem of `which` into out[i][2..7] (entries 0
// and 1 are the probe features and stay untouched).
int density_features(Batch* b, const std::vector<int>& which, const double* const* rho_d, double p, double rho0,
                     std::vector<std::array<float, 8>>& out, hipStream_t s) {
  if (!(p > 0) || !std::isfinite(p)) return fail(TG_EINVAL, "SIMP exponent p must be > 0");
  if (!(rho0 > 0 && rho0 <= 1)) return fail(TG_EINVAL, "floor must be in (0, 1]");
  for (int i : which) {
    if (!rho_d[i]) return fail(TG_EINVAL, "NULL density pointer");
    b->grids[i]->desc.ext0 = rho_d[i];
  }
  int rc = batch_upload_desc(b, s);
  if (rc) return rc;
  if ((rc = batch_set_active(b, which, s, true))) return rc;
  TG_HIP(hipMemsetAsync(b->flag_d, 0, sizeof(int) * b->n, s));
  const DevList& el = b->elem[0];
  if (el.n) {
    k_cc_init<<<el.n, 256, 0, s>>>(b->desc_d, el.ptr);
    k_cc_hook<<<el.n, 256, 0, s>>>(b->desc_d, el.ptr, b->flag_d);
    k_cc_root<<<el.n, 256, 0, s>>>(b->desc_d, el.ptr);
    k_cc_mark<<<el.n, 256, 0, s>>>(b->desc_d, el.ptr);
  }
  if (b->prob.n) k_dstats<<<b->prob.n, 256, 0, s>>>(b->desc_d, b->prob.ptr, p, rho0, b->feat_d);
  TG_HIP(hipGetLastError());
  std::vector<double> fh(8 * (size_t)b->n);
  std::vector<int> err(b->n);
  TG_HIP(hipMemcpyAsync(fh.data(), b->feat_d, sizeof(double) * fh.size(), hipMemcpyDeviceToHost, s));
  TG_HIP(hipMemcpyAsync(err.data(), b->flag_d, sizeof(int) * b->n, hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  if (out.size() < (size_t)b->n) out.resize(b->n);
  for (int i : which) {
    if (err[i]) return fail(TG_EINVAL, "connectivity labelling did not settle");
    for (int q = 0; q < 6; ++q) out[i][2 + q] = (float)fh[8 * (size_t)i + q];
  }
  return TG_OK;
}

}  // namespace tg

using namespace tg;

namespace {
size_t al(size_t n) { return (n + 255) & ~(size_t)255; }
size_t mlp_bytes(int max_batch) {
  return 4 * al(sizeof(float) * NPARAM) + al(sizeof(float) * MAX_WAVES * GSTRIDE) +
         al(sizeof(float) * MAX_WAVES) + al(sizeof(float)) + 2 * al(sizeof(float) * 8) +
         al(sizeof(float) * 8 * (size_t)max_batch) + al(sizeof(float) * 4 * (size_t)max_batch) +
         al(sizeof(int) * (size_t)max_batch);
}
}  // namespace

extern "C" {

int tg_mlp_workspace_bytes(int max_batch, size_t* bytes) {
  if (max_batch < 1 || !bytes) return fail(TG_EINVAL, "max_batch must be >= 1");
  *bytes = mlp_bytes(max_batch);
  return TG_OK;
}

int tg_mlp_create(void* ws_d, size_t bytes, int max_batch, tg_mlp** out) {
  if (!out || max_batch < 1) return fail(TG_EINVAL, "bad MLP create arguments");
  if (!ws_d || bytes < mlp_bytes(max_batch)) return fail(TG_EWORKSPACE, "MLP workspace too small");
  if (((uintptr_t)ws_d) & 255) return fail(TG_EINVAL, "workspace must be 256-byte aligned");
  tg_mlp* m = new tg_mlp();
  char* c = (char*)ws_d;
  auto take = [&](size_t n) {
    char* r = c;
    c += al(n);
    return r;
  };
  m->P = (float*)take(sizeof(float) * NPARAM);
  m->M = (float*)take(sizeof(float) * NPARAM);
  m->V = (float*)take(sizeof(float) * NPARAM);
  m->G = (float*)take(sizeof(float) * NPARAM);
  m->part = (float*)take(sizeof(float) * MAX_WAVES * GSTRIDE);
  m->lpart = (float*)take(sizeof(float) * MAX_WAVES);
  m->loss = (float*)take(sizeof(float));
  m->mean = (float*)take(sizeof(float) * 8);
  m->sd = (float*)take(sizeof(float) * 8);
  m->x = (float*)take(sizeof(float) * 8 * (size_t)max_batch);
  m->logits = (float*)take(sizeof(float) * 4 * (size_t)max_batch);
  m->pred = (int*)take(sizeof(int) * (size_t)max_batch);
  m->max_batch = max_batch;
  *out = m;
  return TG_OK;
}

void tg_mlp_destroy(tg_mlp* m) { delete m; }

int tg_mlp_set_params(tg_mlp* m, const float* params_h, const float* mean_h, const float* std_h, void* stream) {
  if (!m || !params_h) return fail(TG_EINVAL, "NULL argument");
  float mu[8], sd[8];
  for (int k = 0; k < 8; ++k) {
    mu[k] = mean_h ? mean_h[k] : 0.f;
    sd[k] = std_h ? std_h[k] : 1.f;
    if (!(sd[k] > 0.f) || !std::isfinite(sd[k]) || !std::isfinite(mu[k]))
      return fail(TG_EINVAL, "standardization scales must be finite and > 0");
  }
  for (int i = 0; i < NPARAM; ++i)
    if (!std::isfinite(params_h[i])) return fail(TG_EINVAL, "parameters must be finite");
  hipStream_t s = (hipStream_t)stream;
  TG_HIP(hipMemcpyAsync(m->P, params_h, sizeof(float) * NPARAM, hipMemcpyHostToDevice, s));
  TG_HIP(hipMemcpyAsync(m->mean, mu, sizeof(mu), hipMemcpyHostToDevice, s));
  TG_HIP(hipMemcpyAsync(m->sd, sd, sizeof(sd), hipMemcpyHostToDevice, s));
  TG_HIP(hipMemsetAsync(m->M, 0, sizeof(float) * NPARAM, s));
  TG_HIP(hipMemsetAsync(m->V, 0, sizeof(float) * NPARAM, s));
  TG_HIP(hipStreamSynchronize(s));
  m->t = 0;
  m->params_set = true;
  return TG_OK;
}

int tg_mlp_get_params(const tg_mlp* m, float* params_h, void* stream) {
  int rc = mlp_check(m);
  if (rc) return rc;
  if (!params_h) return fail(TG_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  TG_HIP(hipMemcpyAsync(params_h, m->P, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  return TG_OK;
}

int tg_mlp_forward(const tg_mlp* m, const float* x_d, int B, float* logits_d, void* stream) {
  int rc = mlp_check(m);
  if (rc) return rc;
  if (B < 0 || (B > 0 && (!x_d || !logits_d))) return fail(TG_EINVAL, "bad forward arguments");
  return fwd_launch(m, x_d, B, logits_d, nullptr, (hipStream_t)stream);
}

int tg_mlp_train_step(tg_mlp* m, const float* x_d, const int* y_d, int B, float lr, float* loss_h, float* grads_d,
                      void* stream) {
  int rc = mlp_check(m);
  if (rc) return rc;
  if (B < 1 || !x_d || !y_d) return fail(TG_EINVAL, "train step needs B >= 1 samples and labels");
  if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(TG_EINVAL, "learning rate must be finite and >= 0");
  hipStream_t s = (hipStream_t)stream;
  const int waves = std::min(MAX_WAVES, std::max(4, (B + 3) / 4 * 4));
  const int blocks = waves / 4;
  const float invB = 1.0f / (float)B;
  k_mlp_grad<<<blocks, 256, 0, s>>>(m->P, m->mean, m->sd, x_d, y_d, B, invB, m->part, m->lpart);
  TG_HIP(hipGetLastError());
  const long long t = m->t + 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)t)));
  k_mlp_adam<<<(NPARAM + 1 + 255) / 256, 256, 0, s>>>(m->part, m->lpart, blocks * 4, invB, lr, (float)b1, (float)b2,
                                                     1e-8f, c1, c2, 1, m->P, m->M, m->V, m->G, m->loss);
  TG_HIP(hipGetLastError());
  m->t = t;
  if (grads_d) TG_HIP(hipMemcpyAsync(grads_d, m->G, sizeof(float) * NPARAM, hipMemcpyDeviceToDevice, s));
  if (loss_h) {
    TG_HIP(hipMemcpyAsync(loss_h, m->loss, sizeof(float), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
  }
  return TG_OK;
}

int tg_density_features(tg_grid* g, const double* rho_d, double p, double rho0, double* stats_h, void* stream) {
  if (!g || !g->bound) return fail(TG_ESTATE, "grid has no bound workspace");
  if (!rho_d || !stats_h) return fail(TG_EINVAL, "NULL argument");
  std::vector<std::array<float, 8>> f(1);
  const double* r[1] = {rho_d};
  int rc = density_features(g->self, {0}, r, p, rho0, f, (hipStream_t)stream);
  if (rc) return rc;
  // full-precision copy of the statistics
  hipStream_t s = (hipStream_t)stream;
  TG_HIP(hipMemcpyAsync(stats_h, g->self->feat_d, sizeof(double) * 6, hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  return TG_OK;
}

}  // extern "C"
