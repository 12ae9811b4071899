// Device kernels of the guarded SIMP state solve (gfx950).
//
// All kernels take the batch descriptor array and a work list; workgroup b
// serves problem work[b].x, tile work[b].y.  Vectors are full length
// (3 * nodes, AoS) and hold zeros on the clamped x = 0 nodes.
#include <climits>
#include <mutex>

#include "tg_internal.h"

namespace tg {

// ---------------------------------------------------------------------------
// small device helpers
template <class T> __device__ __forceinline__ T* pool(const LevelDesc& L);
template <> __device__ __forceinline__ double* pool<double>(const LevelDesc& L) { return L.vec64; }
template <> __device__ __forceinline__ float* pool<float>(const LevelDesc& L) { return L.vec32; }

// slot >= 0: slot of the pool of type T at this level; slot < 0: external pointer
template <class T>
__device__ __forceinline__ T TG_GLOBAL* vslot(const LevelDesc& L, int slot, const void* ext) {
  return gp(slot < 0 ? (T*)ext : pool<T>(L) + (long long)slot * L.stride);
}
template <class T> __device__ __forceinline__ const T* Dinv(const LevelDesc& L);
template <> __device__ __forceinline__ const double* Dinv<double>(const LevelDesc& L) { return L.Dinv64; }
template <> __device__ __forceinline__ const float* Dinv<float>(const LevelDesc& L) { return L.Dinv32; }
template <class T> __device__ __forceinline__ const T* CinvP(const ProbDesc& P);
template <> __device__ __forceinline__ const double* CinvP<double>(const ProbDesc& P) { return P.Cinv64; }
template <> __device__ __forceinline__ const float* CinvP<float>(const ProbDesc& P) { return P.Cinv32; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sixteen wave sums at once: each butterfly stage pairs a lane with its
// partner across one lane bit and keeps half of the values, so 15 exchanges
// leave every lane with one value summed over 16 lanes, and two more finish the
// sum over the wave.  Lane l < 16 returns the total of value rev4(l), where
// rev4 reverses the four low bits (a fixed order: deterministic).
template <int H, int M>
__device__ __forceinline__ void sum16_stage(double* v, int lane) {
  const bool up = lane & M;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double keep = up ? v[i + H] : v[i];
    const double send = up ? v[i] : v[i + H];
    v[i] = keep + __shfl_xor(send, M, 64);
  }
}
__device__ __forceinline__ double wave_sum16(double* v, int lane) {
  sum16_stage<8, 1>(v, lane);
  sum16_stage<4, 2>(v, lane);
  sum16_stage<2, 4>(v, lane);
  sum16_stage<1, 8>(v, lane);
  double r = v[0];
  r += __shfl_xor(r, 16, 64);
  r += __shfl_xor(r, 32, 64);
  return r;
}
__device__ __forceinline__ int rev4(int l) {
  return ((l & 1) << 3) | ((l & 2) << 1) | ((l & 4) >> 1) | ((l & 8) >> 3);
}

// Deterministic block sum over 256 threads (4 waves); result valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// set_density: E_e = rho_min + (1 - rho_min) rho^p   (Eq. floor_scaling)
__global__ __launch_bounds__(256) void k_young(const ProbDesc* __restrict__ probs,
                                               const int2* __restrict__ work, double p,
                                               int* __restrict__ bad) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& L = P.lv[0];
  const long long n_e = (long long)L.ex * L.ey * L.ez;
  const long long e = (long long)wi.y * 256 + threadIdx.x;
  if (e >= n_e) return;
  const double r = P.ext0[e];
  if (!(r >= 0.0 && r <= 1.0)) {   // also catches NaN
    atomicOr(bad + wi.x, 1);
  }
  const double rc = fmin(fmax(r, 0.0), 1.0);
  const double E = P.rho_min + (1.0 - P.rho_min) * pow(rc, p);
  P.E64[e] = E;
  P.E32[e] = (float)E;
}

// Level-1 Galerkin element matrices: Kel1[C] = sum_c E[child c] * G_c, where
// G_c = P_c^T Ke P_c and P_c interpolates the coarse element's 24 DOFs to
// those of child c (trilinear, exact for nested hex8 spaces).
__global__ __launch_bounds__(256) void k_galerkin1(const ProbDesc* __restrict__ probs,
                                                   const int2* __restrict__ work) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& Lf = P.lv[0];
  const LevelDesc& Lc = P.lv[1];
  const long long C = wi.y;   // one coarse element per workgroup
  const int cx = (int)(C % Lc.ex);
  const int cy = (int)((C / Lc.ex) % Lc.ey);
  const int cz = (int)(C / ((long long)Lc.ex * Lc.ey));
  double Ec[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int fx = 2 * cx + (c & 1), fy = 2 * cy + ((c >> 1) & 1), fz = 2 * cz + ((c >> 2) & 1);
    Ec[c] = P.E64[fx + (long long)Lf.ex * (fy + (long long)Lf.ey * fz)];
  }
  for (int q = threadIdx.x; q < 576; q += 256) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += Ec[c] * P.G64[c * 576 + q];
    Lc.Kel64[C * 576 + q] = s;
  }
}

// Level l -> l+1 (l >= 1): Kel_{l+1}[C] = sum_c P_c^T Kel_l[child c] P_c.
// Each P_c is a scalar trilinear weight matrix W_c (child node a, parent node
// A) times I_3, so both products sum over the 8 nodes of a component, not
// over 24 DOFs: T = Kel_child (W_c x I3), out += (W_c^T x I3) T.
__global__ __launch_bounds__(256) void k_galerkin_up(const ProbDesc* __restrict__ probs,
                                                     const int2* __restrict__ work, int lc) {
  __shared__ double sK[576];
  __shared__ double sT[576];
  __shared__ double sW[64];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& Lf = P.lv[lc - 1];
  const LevelDesc& Lc = P.lv[lc];
  const long long C = wi.y;
  const int cx = (int)(C % Lc.ex);
  const int cy = (int)((C / Lc.ex) % Lc.ey);
  const int cz = (int)(C / ((long long)Lc.ex * Lc.ey));
  double acc[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < 8; ++c) {
    const int fx = 2 * cx + (c & 1), fy = 2 * cy + ((c >> 1) & 1), fz = 2 * cz + ((c >> 2) & 1);
    const long long fe = fx + (long long)Lf.ex * (fy + (long long)Lf.ey * fz);
    // child matrix and its node weights (the x-component entries of P_c)
    for (int q = threadIdx.x; q < 576; q += 256) sK[q] = Lf.Kel64[fe * 576 + q];
    if (threadIdx.x < 64) {
      const int a = threadIdx.x >> 3, A = threadIdx.x & 7;
      sW[threadIdx.x] = P.Pc64[c * 576 + (3 * a) * 24 + 3 * A];
    }
    __syncthreads();
    // T[r][3A + j] = sum_a Kel[r][3a + j] W[a][A]
    for (int q = threadIdx.x; q < 576; q += 256) {
      const int r = q / 24, col = q % 24, A = col / 3, j = col % 3;
      double t = 0.0;
#pragma unroll
      for (int a = 0; a < 8; ++a) t += sK[r * 24 + 3 * a + j] * sW[a * 8 + A];
      sT[q] = t;
    }
    __syncthreads();
    // out[3B + i][col] += sum_b W[b][B] T[3b + i][col]
    int qq = 0;
    for (int q = threadIdx.x; q < 576; q += 256, ++qq) {
      const int row = q / 24, col = q % 24, B = row / 3, i = row % 3;
      double t = 0.0;
#pragma unroll
      for (int bb = 0; bb < 8; ++bb) t += sW[bb * 8 + B] * sT[(3 * bb + i) * 24 + col];
      acc[qq] += t;
    }
    __syncthreads();
  }
  int qq = 0;
  for (int q = threadIdx.x; q < 576; q += 256, ++qq) Lc.Kel64[C * 576 + q] = acc[qq];
}

// Mode-basis form of the level-l Galerkin element matrices (l > TG_MF_LEVELS):
// Khat = H Kel H^T / 64 with H the per-component 8-point +-1 transform of
// the node index (DOF 3 a + c -> 3 m + c, H[m][a] = prod over the bits b of m
// of (2 bit_b(a) - 1)), symmetrized, and its TG_GM_NU pattern entries stored
// at Km[e * TG_GM_STRIDE + v] (padding zero).  Entries off the pattern vanish
// in exact arithmetic.
__global__ __launch_bounds__(256) void k_mode_pack(const ProbDesc* __restrict__ probs,
                                                   const int2* __restrict__ work, int l) {
  __shared__ double sK[576];
  __shared__ double sX[576];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& L = P.lv[l];
  const long long e = wi.y;   // one element per workgroup
  auto H = [](int m, int a) { return (__popc(m & ~a) & 1) ? -1.0 : 1.0; };
  for (int q = threadIdx.x; q < 576; q += 256) sK[q] = L.Kel64[e * 576 + q];
  __syncthreads();
  // X = (H x I3) Kel
  for (int q = threadIdx.x; q < 576; q += 256) {
    const int r = q / 24, c = q % 24, m = r / 3, i = r % 3;
    double t = 0.0;
    for (int a = 0; a < 8; ++a) t += H(m, a) * sK[(3 * a + i) * 24 + c];
    sX[q] = t;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < TG_GM_STRIDE; v += 256) {
    if (v >= TG_GM_NU) {
      L.Km64[gm_index(e, v, 2)] = 0.0;
      L.Km32[gm_index(e, v, 4)] = 0.f;
      continue;
    }
    const int r = kGMPairs[v][0], c = kGMPairs[v][1];
    // Khat[r][c] = sum_b X[r][3 b + j] H[n][b] / 64, and its transpose
    const int n = c / 3, j = c % 3, m = r / 3, i = r % 3;
    double t1 = 0.0, t2 = 0.0;
    for (int b = 0; b < 8; ++b) {
      t1 += sX[r * 24 + 3 * b + j] * H(n, b);
      t2 += sX[c * 24 + 3 * b + i] * H(m, b);
    }
    const double k = 0.5 * (t1 + t2) / 64.0;
    L.Km64[gm_index(e, v, 2)] = k;
    L.Km32[gm_index(e, v, 4)] = (float)k;
  }
}

// Node-block diagonal (3x3, coupling u_x, u_y, u_z of one node) and its inverse.
__global__ __launch_bounds__(256) void k_nodeblock(const ProbDesc* __restrict__ probs,
                                                   const int2* __restrict__ work, int l) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& L = P.lv[l];
  const int n = wi.y * TG_NODE_TILE + threadIdx.x;
  if (n >= L.n_nodes) return;
  const int i = n % L.NX, t = n / L.NX, j = t % L.NY, k = t / L.NY;
  double B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int a = 0; a < 8; ++a) {
    const int ex = i - (a & 1), ey = j - ((a >> 1) & 1), ez = k - ((a >> 2) & 1);
    if (ex < 0 || ex >= L.ex || ey < 0 || ey >= L.ey || ez < 0 || ez >= L.ez) continue;
    const long long e = ex + (long long)L.ex * (ey + (long long)L.ey * ez);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const int q = (3 * a + r) * 24 + 3 * a + c;
        B[3 * r + c] += (l == 0) ? P.E64[e] * P.Ke64[q] : L.Kel64[e * 576 + q];
      }
  }
  double D[9];
  if (i == 0) {
    for (int q = 0; q < 9; ++q) D[q] = (q % 4 == 0) ? 1.0 : 0.0;
  } else {
    const double c00 = B[4] * B[8] - B[5] * B[7];
    const double c01 = B[5] * B[6] - B[3] * B[8];
    const double c02 = B[3] * B[7] - B[4] * B[6];
    const double det = B[0] * c00 + B[1] * c01 + B[2] * c02;
    const double id = 1.0 / det;
    D[0] = c00 * id;
    D[1] = (B[2] * B[7] - B[1] * B[8]) * id;
    D[2] = (B[1] * B[5] - B[2] * B[4]) * id;
    D[3] = c01 * id;
    D[4] = (B[0] * B[8] - B[2] * B[6]) * id;
    D[5] = (B[2] * B[3] - B[0] * B[5]) * id;
    D[6] = c02 * id;
    D[7] = (B[1] * B[6] - B[0] * B[7]) * id;
    D[8] = (B[0] * B[4] - B[1] * B[3]) * id;
  }
  for (int q = 0; q < 9; ++q) {
    L.Dinv64[9LL * n + q] = D[q];
    L.Dinv32[9LL * n + q] = (float)D[q];
  }
}

// Coarsest level: assemble the dense free-DOF matrix, Cholesky-factor it and
// form the explicit inverse (one workgroup per problem).
__device__ __forceinline__ int coarse_free_index(const LevelDesc& L, int node, int c) {
  const int i = node % L.NX, t = node / L.NX;   // t = j + NY k
  return i == 0 ? -1 : 3 * ((L.NX - 1) * t + (i - 1)) + c;
}

__global__ __launch_bounds__(256) void k_coarse_factor(const ProbDesc* __restrict__ probs,
                                                       const int2* __restrict__ work, int* bad, int nmin) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const int l = P.nlev - 1;
  const LevelDesc& L = P.lv[l];
  const int n = P.ncoarse;
  if (n == 0 || n < nmin) return;  // no direct-solvable coarsest level, or one k_coarse_factor_lds took
  double* A = P.Cwork;             // n x n, row-major; lower triangle -> L
  double* X = P.Cwork + (long long)n * n;
  for (int q = threadIdx.x; q < n * n; q += blockDim.x) A[q] = 0.0;
  __syncthreads();
  const int ne = L.ex * L.ey * L.ez;
  for (int e = 0; e < ne; ++e) {
    const int ex = e % L.ex, ey = (e / L.ex) % L.ey, ez = e / (L.ex * L.ey);
    for (int q = threadIdx.x; q < 576; q += blockDim.x) {
      const int r = q / 24, c = q % 24;
      const int a = r / 3, b = c / 3;
      const int na = (ex + (a & 1)) + L.NX * ((ey + ((a >> 1) & 1)) + L.NY * (ez + ((a >> 2) & 1)));
      const int nb = (ex + (b & 1)) + L.NX * ((ey + ((b >> 1) & 1)) + L.NY * (ez + ((b >> 2) & 1)));
      const int fr = coarse_free_index(L, na, r % 3), fc = coarse_free_index(L, nb, c % 3);
      if (fr < 0 || fc < 0) continue;
      const double v = (l == 0) ? P.E64[e] * P.Ke64[q] : L.Kel64[(long long)e * 576 + q];
      A[fr * n + fc] += v;         // distinct (fr, fc) within one element
    }
    __syncthreads();
  }
  // right-looking Cholesky, lower triangle
  __shared__ double piv;
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      const double d = A[k * n + k];
      if (!(d > 0.0)) atomicOr(bad + wi.x, 2);
      piv = sqrt(fmax(d, 1e-300));
      A[k * n + k] = piv;
    }
    __syncthreads();
    for (int r = k + 1 + threadIdx.x; r < n; r += blockDim.x) A[r * n + k] /= piv;
    __syncthreads();
    for (int q = threadIdx.x; q < (n - k - 1) * (n - k - 1); q += blockDim.x) {
      const int r = k + 1 + q / (n - k - 1), c = k + 1 + q % (n - k - 1);
      if (c <= r) A[r * n + c] -= A[r * n + k] * A[c * n + k];
    }
    __syncthreads();
  }
  // inverse: column q of X solves L L^T x = e_q (one column per thread)
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    for (int r = 0; r < n; ++r) {     // forward: L y = e_q
      double s = (r == q) ? 1.0 : 0.0;
      for (int c = q; c < r; ++c) s -= A[r * n + c] * X[c * n + q];
      X[r * n + q] = (r < q) ? 0.0 : s / A[r * n + r];
    }
    for (int r = n - 1; r >= 0; --r) {   // backward: L^T x = y
      double s = X[r * n + q];
      for (int c = r + 1; c < n; ++c) s -= A[c * n + r] * X[c * n + q];
      X[r * n + q] = s / A[r * n + r];
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
    const int r = q / n, c = q % n;
    // symmetrize the explicit inverse
    const double v = 0.5 * (X[r * n + c] + X[c * n + r]);
    P.Cinv64[q] = v;
    P.Cinv32[q] = (float)v;
  }
}

// The same coarsest-level set-up held in LDS, for coarsest levels whose
// matrix fits (n^2 + 2 n doubles): the assembled matrix is inverted in place
// by Gauss-Jordan elimination without pivoting (its pivots are the diagonal
// entries of successive Schur complements, positive for an SPD matrix), all
// n^2 updates of a step in parallel; the explicit inverse is symmetrized as
// in k_coarse_factor.  A non-positive pivot flags the problem.
#define CF_THREADS 1024
#define CF_REG 16   // register form: rows per thread (n <= 128)
__global__ __launch_bounds__(CF_THREADS) void k_coarse_factor_lds(const ProbDesc* __restrict__ probs,
                                                                  const int2* __restrict__ work, int* bad,
                                                                  int nmax) {
  extern __shared__ double smem[];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const int l = P.nlev - 1;
  const LevelDesc& L = P.lv[l];
  const int n = P.ncoarse;
  if (n == 0 || n > nmax) return;   // larger coarsest levels: k_coarse_factor
  double* A = smem;                  // n x n, row-major
  double* rowk = smem + n * n;       // pivot row, scaled
  double* colk = rowk + n;           // pivot column
  for (int q = threadIdx.x; q < n * n; q += blockDim.x) A[q] = 0.0;
  __syncthreads();
  const int ne = L.ex * L.ey * L.ez;
  for (int e = 0; e < ne; ++e) {
    const int ex = e % L.ex, ey = (e / L.ex) % L.ey, ez = e / (L.ex * L.ey);
    for (int q = threadIdx.x; q < 576; q += blockDim.x) {
      const int r = q / 24, c = q % 24;
      const int a = r / 3, b = c / 3;
      const int na = (ex + (a & 1)) + L.NX * ((ey + ((a >> 1) & 1)) + L.NY * (ez + ((a >> 2) & 1)));
      const int nb = (ex + (b & 1)) + L.NX * ((ey + ((b >> 1) & 1)) + L.NY * (ez + ((b >> 2) & 1)));
      const int fr = coarse_free_index(L, na, r % 3), fc = coarse_free_index(L, nb, c % 3);
      if (fr < 0 || fc < 0) continue;
      const double v = (l == 0) ? P.E64[e] * P.Ke64[q] : L.Kel64[(long long)e * 576 + q];
      A[fr * n + fc] += v;         // distinct (fr, fc) within one element
    }
    __syncthreads();
  }
  // Register form: thread t holds column j = t mod n of the rows t / n +
  // q rpp (rpp = rows per pass, q < cm).  Each step publishes the pivot
  // column and row through one of two alternating LDS buffers (one barrier
  // per step); the column is stored in slot order, row i at
  // (i mod rpp) cm + i / rpp, so a thread's rows are contiguous.  Every
  // register takes the generic update a -= c_i r_j / p (unused ones too, on
  // values never stored), then the holders of row k and of column k write
  // their special values: the same operations as the LDS form below.
  const int rpp = CF_THREADS / n;
  const int cm = (n + rpp - 1) / rpp;
  if (n >= 2 && cm <= CF_REG) {
    const int t = threadIdx.x, j = t % n, i0 = t / n;
    const bool act = t < rpp * n;
    const int cnt = act ? (n - i0 + rpp - 1) / rpp : 0;
    const int csz = rpp * cm + CF_REG, bsz = csz + n;   // column part (padded), buffer
    const int cb = (act ? i0 : 0) * cm;                 // this thread's first slot
    double a[CF_REG];
#pragma unroll
    for (int q = 0; q < CF_REG; ++q) a[q] = q < cnt ? A[(i0 + q * rpp) * n + j] : 0.0;
    __syncthreads();   // A's storage now holds the pivot buffers
    for (int k = 0; k < n; ++k) {
      double* ck = smem + (k & 1) * bsz;
      double* rk = ck + csz;
      const bool rowk = act && k % rpp == i0, colk = act && j == k;
      const int qk = k / rpp;
      if (colk) {
#pragma unroll
        for (int q = 0; q < CF_REG; ++q)
          if (q < cnt) ck[cb + q] = a[q];
      }
      if (rowk) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < CF_REG; ++q) v = q == qk ? a[q] : v;
        rk[j] = v;
      }
      __syncthreads();
      const double p = ck[(k % rpp) * cm + qk];
      if (t == 0 && !(p > 0.0)) atomicOr(bad + wi.x, 2);
      const double ip = 1.0 / p;
      const double rj = rk[j] * ip;
      double ci[CF_REG];
#pragma unroll
      for (int q = 0; q < CF_REG; ++q) ci[q] = ck[cb + q];
#pragma unroll
      for (int q = 0; q < CF_REG; ++q) a[q] -= ci[q] * rj;
      if (rowk) {
        const double v = colk ? ip : rj;
#pragma unroll
        for (int q = 0; q < CF_REG; ++q) a[q] = q == qk ? v : a[q];
      }
      if (colk) {
#pragma unroll
        for (int q = 0; q < CF_REG; ++q)
          if (q < cnt && i0 + q * rpp != k) a[q] = -ci[q] * ip;
      }
    }
    __syncthreads();   // every read of the last pivot buffers is done
#pragma unroll
    for (int q = 0; q < CF_REG; ++q)
      if (q < cnt) A[(i0 + q * rpp) * n + j] = a[q];
    __syncthreads();
  } else {
  for (int k = 0; k < n; ++k) {
    const double p = A[k * n + k];
    if (threadIdx.x == 0 && !(p > 0.0)) atomicOr(bad + wi.x, 2);
    const double ip = 1.0 / p;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      colk[j] = A[j * n + k];
      rowk[j] = A[k * n + j] * ip;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
      const int i = q / n, j = q - (q / n) * n;
      if (i == k)
        A[q] = (j == k) ? ip : rowk[j];
      else if (j == k)
        A[q] = -colk[i] * ip;
      else
        A[q] -= colk[i] * rowk[j];
    }
    __syncthreads();
  }
  }
  for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
    const int r = q / n, c = q % n;
    const double v = 0.5 * (A[r * n + c] + A[c * n + r]);
    P.Cinv64[q] = v;
    P.Cinv32[q] = (float)v;
  }
}

// ---------------------------------------------------------------------------
// Operator modes of the level kernels (the z-march kernels of tg_fine.hip):
//   OP_APPLY : y = K x
//   OP_RESID : y = b - K x
//   OP_SMOOTH: y = x + w D^-1 (b - K x)      (damped node-block Jacobi)
//   OP_RESTRICT: b_{l+1} = P^T (b - K x)     (residual fused with the restriction)
//   OP_SMOOTH1: level 0, the first two sweeps from x = 0 with b read from an
//               FP64 slot (x = scale offset, y2 = slot of b's FP32 copy)
enum { OP_APPLY = 0, OP_RESID = 1, OP_SMOOTH = 2, OP_RESTRICT = 3, OP_SMOOTH1 = 4 };

// First pre-sweep from x = 0: x = w D^-1 b; optionally keep b in type T.
template <class TB, class T>
__global__ __launch_bounds__(256) void k_jacobi_first(const ProbDesc* __restrict__ probs,
                                                      const int2* __restrict__ work, int l, int sb,
                                                      const void* eb_, int sbT, int sx, T omega,
                                                      int scale_off) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const LevelDesc& L = P.lv[l];
  const int n = wi.y * TG_NODE_TILE + threadIdx.x;
  if (n >= L.n_nodes) return;
  const auto* b = vslot<TB>(L, sb, eb_);
  auto* x = vslot<T>(L, sx, nullptr);
  // optional per-problem input scale (small[scale_off]), applied in FP64
  const double sc = scale_off >= 0 ? P.small[scale_off] : 1.0;
  T b0 = T(double(b[3LL * n]) * sc), b1 = T(double(b[3LL * n + 1]) * sc), b2 = T(double(b[3LL * n + 2]) * sc);
  if (n % L.NX == 0) b0 = b1 = b2 = T(0);
  if (sbT != INT_MIN) {
    auto* bT = vslot<T>(L, sbT, nullptr);
    bT[3LL * n] = b0;
    bT[3LL * n + 1] = b1;
    bT[3LL * n + 2] = b2;
  }
  const T* D = Dinv<T>(L) + 9LL * n;
  x[3LL * n] = omega * (D[0] * b0 + D[1] * b1 + D[2] * b2);
  x[3LL * n + 1] = omega * (D[3] * b0 + D[4] * b1 + D[5] * b2);
  x[3LL * n + 2] = omega * (D[6] * b0 + D[7] * b1 + D[8] * b2);
}

// Prolongation and correction x_f += P e_c (trilinear); slots < 0 take the
// external vectors ee (coarse) and ex (fine).
template <class T>
__global__ __launch_bounds__(256) void k_prolong(const ProbDesc* __restrict__ probs,
                                                 const int2* __restrict__ work, int l, int sx,
                                                 int se, const void* ee, void* ex, int vbskip) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  if (vbskip && l >= (sizeof(T) == 8 ? P.vb_lb64 : P.vb_lb32)) return;   // run by k_vbottom
  const LevelDesc& Lf = P.lv[l];
  const LevelDesc& Lc = P.lv[l + 1];
  const int n = wi.y * TG_NODE_TILE + threadIdx.x;
  if (n >= Lf.n_nodes) return;
  const int i = n % Lf.NX, t = n / Lf.NX, j = t % Lf.NY, k = t / Lf.NY;
  if (i == 0) return;
  const auto* e = vslot<T>(Lc, se, ee);
  auto* x = vslot<T>(Lf, sx, ex);
  const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
  const T wi_ = (i & 1) ? T(0.5) : T(1), wj = (j & 1) ? T(0.5) : T(1), wk = (k & 1) ? T(0.5) : T(1);
  T s0 = T(0), s1 = T(0), s2 = T(0);
  for (int c = 0; c < 8; ++c) {
    if ((c & 1) && !(i & 1)) continue;
    if ((c & 2) && !(j & 1)) continue;
    if ((c & 4) && !(k & 1)) continue;
    const int I = (c & 1) ? i1 : i0, J = (c & 2) ? j1 : j0, K = (c & 4) ? k1 : k0;
    const long long m = I + (long long)Lc.NX * (J + (long long)Lc.NY * K);
    const T w = wi_ * wj * wk;
    s0 += w * e[3 * m];
    s1 += w * e[3 * m + 1];
    s2 += w * e[3 * m + 2];
  }
  x[3LL * n] += s0;
  x[3LL * n + 1] += s1;
  x[3LL * n + 2] += s2;
}

// Coarsest solve x = K_c^-1 b with the explicit inverse (one workgroup per problem).
template <class TB, class T, class TY>
__global__ __launch_bounds__(256) void k_coarse_solve(const ProbDesc* __restrict__ probs,
                                                      const int2* __restrict__ work, int l, int sb,
                                                      const void* eb_, int sy, void* ey_, int vbskip) {
  __shared__ T sb_[TG_MAX_COARSE];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  if (vbskip && l >= (sizeof(TY) == 8 ? P.vb_lb64 : P.vb_lb32)) return;   // run by k_vbottom
  const LevelDesc& L = P.lv[l];
  const int n = P.ncoarse;
  const auto* b = vslot<TB>(L, sb, eb_);
  auto* y = vslot<TY>(L, sy, ey_);
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const int c = q % 3, fn = q / 3;
    const int i = fn % (L.NX - 1) + 1, t = fn / (L.NX - 1);
    sb_[q] = T(b[3LL * (i + (long long)L.NX * t) + c]);
  }
  __syncthreads();
  const T* Ci = CinvP<T>(P);
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    T s = T(0);
    for (int c = 0; c < n; ++c) s += Ci[(long long)q * n + c] * sb_[c];
    const int cc = q % 3, fn = q / 3;
    const int i = fn % (L.NX - 1) + 1, t = fn / (L.NX - 1);
    y[3LL * (i + (long long)L.NX * t) + cc] = TY(s);
  }
  for (int node = threadIdx.x; node < L.n_nodes; node += blockDim.x) {
    if (node % L.NX == 0) {
      y[3LL * node] = TY(0);
      y[3LL * node + 1] = TY(0);
      y[3LL * node + 2] = TY(0);
    }
  }
}

// Copy between typed vectors at one level (masking the clamped nodes).
template <class TA, class TB>
__global__ __launch_bounds__(256) void k_copy_level(const ProbDesc* __restrict__ probs,
                                                    const int2* __restrict__ work, int l, int sa,
                                                    const void* ea, int sb, void* eb, int scale_off) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const LevelDesc& L = P.lv[l];
  const int n = wi.y * TG_NODE_TILE + threadIdx.x;
  if (n >= L.n_nodes) return;
  const auto* a = vslot<TA>(L, sa, ea);
  auto* b = vslot<TB>(L, sb, eb);
  const bool clamp = (n % L.NX) == 0;
  const double sc = scale_off >= 0 ? P.small[scale_off] : 1.0;
  for (int c = 0; c < 3; ++c) b[3LL * n + c] = clamp ? TB(0) : TB(double(a[3LL * n + c]) * sc);
}

// ---------------------------------------------------------------------------
// Vector kernels on the level-0 FP64 pool (work list: {problem, chunk}).
__device__ __forceinline__ void chunk_range(const LevelDesc& L, int c, long long& lo, long long& hi) {
  lo = (long long)c * TG_VCHUNK;
  hi = lo + TG_VCHUNK;
  const long long n = 3LL * L.n_nodes;
  if (hi > n) hi = n;
}

// dir 0: slot <- ext0 (masked); dir 1: ext1 <- slot
__global__ __launch_bounds__(256) void k_copy_ext_(const ProbDesc* __restrict__ probs,
                                                   const int2* __restrict__ work, int dir, int slot) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& L = P.lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  auto* v = gp(L.vec64 + (long long)slot * L.stride);
  for (long long q = lo + threadIdx.x; q < hi; q += 256) {
    if (dir == 0) {
      const long long node = q / 3;
      v[q] = (node % L.NX == 0) ? 0.0 : P.ext0[q];
    } else {
      P.ext1[q] = v[q];
    }
  }
}

__global__ __launch_bounds__(256) void k_fill0_(const ProbDesc* __restrict__ probs,
                                                const int2* __restrict__ work, int slot, double val) {
  const int2 wi = work[blockIdx.x];
  const LevelDesc& L = probs[wi.x].lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  auto* v = gp(L.vec64 + (long long)slot * L.stride);
  for (long long q = lo + threadIdx.x; q < hi; q += 256) v[q] = val;
}

__global__ __launch_bounds__(256) void k_copy0_(const ProbDesc* __restrict__ probs,
                                                const int2* __restrict__ work, int src, int dst) {
  const int2 wi = work[blockIdx.x];
  const LevelDesc& L = probs[wi.x].lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  const auto* a = gp(L.vec64 + (long long)src * L.stride);
  auto* b = gp(L.vec64 + (long long)dst * L.stride);
  for (long long q = lo + threadIdx.x; q < hi; q += 256) b[q] = a[q];
}

// Partial dots: part[k * n_chunks + chunk] = sum_{q in chunk} V_{sbase+k}[q] * w[q]
// for k < nv; if with_self, entry nv holds w . w.
__global__ __launch_bounds__(256) void k_multidot_(const ProbDesc* __restrict__ probs,
                                                   const int2* __restrict__ work, int sbase, int nv,
                                                   int sw, int with_self) {
  __shared__ double sh[8][4];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const LevelDesc& L = P.lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  const auto* w = gp(L.vec64 + (long long)sw * L.stride);
  double wr[TG_VCHUNK / 256];
#pragma unroll
  for (int q = 0; q < TG_VCHUNK / 256; ++q) {
    const long long idx = lo + threadIdx.x + 256LL * q;
    wr[q] = idx < hi ? w[idx] : 0.0;
  }
  const int ntot = nv + (with_self ? 1 : 0);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k0 = 0; k0 < ntot; k0 += 8) {
    double s[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      s[g] = 0.0;
      const int k = k0 + g;
      if (k < ntot) {
        const auto* v = (k < nv) ? gp(L.vec64 + (long long)(sbase + k) * L.stride) : w;
#pragma unroll
        for (int q = 0; q < TG_VCHUNK / 256; ++q) {
          const long long idx = lo + threadIdx.x + 256LL * q;
          if (idx < hi) s[g] += v[idx] * wr[q];
        }
      }
    }
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const double r = wave_sum(s[g]);
      if (lane == 0) sh[g][wv] = r;
    }
    __syncthreads();
    if (threadIdx.x < 8 && k0 + (int)threadIdx.x < ntot) {
      const int g = threadIdx.x;
      P.part[(long long)(k0 + g) * L.n_chunks + wi.y] = (sh[g][0] + sh[g][1]) + (sh[g][2] + sh[g][3]);
    }
    __syncthreads();
  }
}

// tmp[dst + k] = sum over chunks of part[k][.] in a fixed order.  mode 0 also
// assigns h[k], mode 1 adds into h[k], mode 2 touches only tmp.  Entry k ==
// save_k (if >= 0) goes to scal[SC_FLAG] instead.  Grid: (problems, nv).
__global__ __launch_bounds__(256) void k_reduce_(const ProbDesc* __restrict__ probs,
                                                 const int2* __restrict__ work, int h_off,
                                                 int tmp_off, int flag_off, int mode, int save_k) {
  __shared__ double sh[4];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const int nc = P.lv[0].n_chunks;
  const int k = blockIdx.y;
  double s = 0.0;
  for (int c = threadIdx.x; c < nc; c += 256) s += P.part[(long long)k * nc + c];
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) {
    if (k == save_k) {
      P.small[flag_off] = s;
      return;
    }
    P.small[tmp_off + k] = s;
    if (mode == 0) P.small[h_off + k] = s;
    if (mode == 1) P.small[h_off + k] += s;
  }
}

// w -= sum_k coef[k] V_{sbase+k}
__global__ __launch_bounds__(256) void k_update_(const ProbDesc* __restrict__ probs,
                                                 const int2* __restrict__ work, int sbase, int nv,
                                                 int sw, int coef_off) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const LevelDesc& L = P.lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  auto* w = gp(L.vec64 + (long long)sw * L.stride);
  const double* coef = P.small + coef_off;
  double acc[TG_VCHUNK / 256];
#pragma unroll
  for (int q = 0; q < TG_VCHUNK / 256; ++q) acc[q] = 0.0;
  for (int k = 0; k < nv; ++k) {
    const double ck = coef[k];
    const auto* v = gp(L.vec64 + (long long)(sbase + k) * L.stride);
#pragma unroll
    for (int q = 0; q < TG_VCHUNK / 256; ++q) {
      const long long idx = lo + threadIdx.x + 256LL * q;
      if (idx < hi) acc[q] += ck * v[idx];
    }
  }
#pragma unroll
  for (int q = 0; q < TG_VCHUNK / 256; ++q) {
    const long long idx = lo + threadIdx.x + 256LL * q;
    if (idx < hi) w[idx] -= acc[q];
  }
}

// Fused Gram-Schmidt sweep: w -= sum_k coef[k] V_k over the chunk, then the
// chunk partials of V_k . w (k < ndot) and, if with_self, of w . w, written
// like k_multidot_.  The update of one chunk only needs that chunk, so the
// dots of the updated vector are exact chunk sums.
__global__ __launch_bounds__(256) void k_update_dots_(const ProbDesc* __restrict__ probs,
                                                      const int2* __restrict__ work, int sbase, int nv,
                                                      int sw, int coef_off, int ndot, int with_self) {
  __shared__ double sh[8][4];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const LevelDesc& L = P.lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  auto* w = gp(L.vec64 + (long long)sw * L.stride);
  const double* coef = P.small + coef_off;
  double wr[TG_VCHUNK / 256];
#pragma unroll
  for (int q = 0; q < TG_VCHUNK / 256; ++q) {
    const long long idx = lo + threadIdx.x + 256LL * q;
    wr[q] = idx < hi ? w[idx] : 0.0;
  }
  {
    double acc[TG_VCHUNK / 256];
#pragma unroll
    for (int q = 0; q < TG_VCHUNK / 256; ++q) acc[q] = 0.0;
    for (int k = 0; k < nv; ++k) {
      const double ck = coef[k];
      const auto* v = gp(L.vec64 + (long long)(sbase + k) * L.stride);
#pragma unroll
      for (int q = 0; q < TG_VCHUNK / 256; ++q) {
        const long long idx = lo + threadIdx.x + 256LL * q;
        if (idx < hi) acc[q] += ck * v[idx];
      }
    }
#pragma unroll
    for (int q = 0; q < TG_VCHUNK / 256; ++q) {
      const long long idx = lo + threadIdx.x + 256LL * q;
      wr[q] -= acc[q];
      if (idx < hi) w[idx] = wr[q];
    }
  }
  const int ntot = ndot + (with_self ? 1 : 0);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k0 = 0; k0 < ntot; k0 += 8) {
    double sacc[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      sacc[g] = 0.0;
      const int k = k0 + g;
      if (k < ntot) {
        if (k < ndot) {
          const auto* v = gp(L.vec64 + (long long)(sbase + k) * L.stride);
#pragma unroll
          for (int q = 0; q < TG_VCHUNK / 256; ++q) {
            const long long idx = lo + threadIdx.x + 256LL * q;
            if (idx < hi) sacc[g] += v[idx] * wr[q];
          }
        } else {
#pragma unroll
          for (int q = 0; q < TG_VCHUNK / 256; ++q) sacc[g] += wr[q] * wr[q];
        }
      }
    }
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const double r = wave_sum(sacc[g]);
      if (lane == 0) sh[g][wv] = r;
    }
    __syncthreads();
    if (threadIdx.x < 8 && k0 + (int)threadIdx.x < ntot) {
      const int g = threadIdx.x;
      P.part[(long long)(k0 + g) * L.n_chunks + wi.y] = (sh[g][0] + sh[g][1]) + (sh[g][2] + sh[g][3]);
    }
    __syncthreads();
  }
}

// Single-read form of the fused sweep for nv <= NVR: each thread keeps its
// DOF's values of all V_k in registers, so V is read once for both the update
// and the dots of the updated vector.
template <int NVR>
__global__ __launch_bounds__(256) void k_update_dots_reg_(const ProbDesc* __restrict__ probs,
                                                          const int2* __restrict__ work, int sbase, int nv,
                                                          int sw, int coef_off, int ndot, int with_self) {
  __shared__ double sh[NVR + 1][4];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const LevelDesc& L = P.lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  auto* w = gp(L.vec64 + (long long)sw * L.stride);
  const auto* V0 = gp(L.vec64 + (long long)sbase * L.stride);
  const long long st = L.stride;
  const double* coef = P.small + coef_off;
  double cf[NVR], acc[NVR + 1];
#pragma unroll
  for (int k = 0; k < NVR; ++k) {
    cf[k] = k < nv ? coef[k] : 0.0;
    acc[k] = 0.0;
  }
  acc[NVR] = 0.0;
  for (int q = 0; q < TG_VCHUNK / 256; ++q) {
    const long long idx = lo + threadIdx.x + 256LL * q;
    if (idx >= hi) break;
    double v[NVR];
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < NVR; ++k) {
      v[k] = k < nv ? V0[k * st + idx] : 0.0;
      t += cf[k] * v[k];
    }
    const double wn = w[idx] - t;
    w[idx] = wn;
#pragma unroll
    for (int k = 0; k < NVR; ++k) acc[k] += v[k] * wn;
    acc[NVR] += wn * wn;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NVR; ++k) {
    if (k < ndot) {
      const double r = wave_sum(acc[k]);
      if (lane == 0) sh[k][wv] = r;
    }
  }
  if (with_self) {
    const double r = wave_sum(acc[NVR]);
    if (lane == 0) sh[NVR][wv] = r;
  }
  __syncthreads();
  const int ntot = ndot + (with_self ? 1 : 0);
  if ((int)threadIdx.x < ntot) {
    const int k = threadIdx.x;
    const int src = k < ndot ? k : NVR;
    P.part[(long long)k * L.n_chunks + wi.y] = (sh[src][0] + sh[src][1]) + (sh[src][2] + sh[src][3]);
  }
}

struct SmallOffs {
  int mmax, H, g, cs, sn, y, h, tmp, scal, hist;
};
// the scalar parts of a delayed-CGS2 step, run by one wave (defined below)
__device__ void dcgs_a_wave(const ProbDesc& P, int p, const SmallOffs& o, int j, double* status_out);
__device__ void dcgs_b_wave(const ProbDesc& P, int p, const SmallOffs& o, int j, int cap, double tol, double brk,
                            double* status_out);

// CGS2 with delayed reorthogonalization, sweep A.  For k < nv the chunk
// partials of V_k . q and V_k . w, then q . q, q . w, w . w: 2 nv + 3 entries
// in the order [V.q (nv) | V.w (nv) | q.q, q.w, w.w].  One read of V, q, w.
__global__ __launch_bounds__(256) void k_dots2_(const ProbDesc* __restrict__ probs,
                                                const int2* __restrict__ work, int sbase, int nv, int sq,
                                                int sw) {
  // per group of eight basis vectors: the 16 wave sums of each wave (every
  // group has its own slots, so the waves only meet once, at the end)
  constexpr int NGRP = (TG_MAX_RESTART + 8) / 8;
  __shared__ double sh[NGRP][16][4];
  __shared__ double sh3[3][4];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const LevelDesc& L = P.lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  const long long nc = L.n_chunks;
  const auto* qv = gp(L.vec64 + (long long)sq * L.stride);
  const auto* wv = gp(L.vec64 + (long long)sw * L.stride);
  // whole chunks: the slot stride is a multiple of the chunk and the tail
  // beyond 3 n_nodes holds zeros
  constexpr int NQ = TG_VCHUNK / 256;
  double qr[NQ], wr[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const long long idx = lo + threadIdx.x + 256LL * q;
    qr[q] = qv[idx];
    wr[q] = wv[idx];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k0 = 0; k0 < nv; k0 += 8) {
    const int gi = k0 >> 3;
    double a[8], c[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      a[g] = c[g] = 0.0;
      const int k = k0 + g;
      if (k < nv) {
        const auto* v = gp(L.vec64 + (long long)(sbase + k) * L.stride);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const double x = v[lo + threadIdx.x + 256LL * q];
          a[g] += x * qr[q];
          c[g] += x * wr[q];
        }
      }
    }
    double v16[16];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      v16[g] = a[g];
      v16[8 + g] = c[g];
    }
    const double r = wave_sum16(v16, lane);
    if (lane < 16) sh[gi][rev4(lane)][wave] = r;
  }
  double qq = 0.0, qw = 0.0, ww = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    qq += qr[q] * qr[q];
    qw += qr[q] * wr[q];
    ww += wr[q] * wr[q];
  }
  qq = wave_sum(qq);
  qw = wave_sum(qw);
  ww = wave_sum(ww);
  if (lane == 0) {
    sh3[0][wave] = qq;
    sh3[1][wave] = qw;
    sh3[2][wave] = ww;
  }
  __syncthreads();
  // rows [V.q | V.w]: row which * nv + k from slot (k & 7) + 8 which of group k / 8
  for (int t = threadIdx.x; t < 2 * nv; t += 256) {
    const int which = t / nv, k = t - which * nv, gi = k >> 3, sl = (k & 7) + 8 * which;
    P.part[(long long)t * nc + wi.y] = (sh[gi][sl][0] + sh[gi][sl][1]) + (sh[gi][sl][2] + sh[gi][sl][3]);
  }
  if (threadIdx.x < 3) {
    const int t = threadIdx.x;
    P.part[(2LL * nv + t) * nc + wi.y] = (sh3[t][0] + sh3[t][1]) + (sh3[t][2] + sh3[t][3]);
  }
}

// CGS2 with delayed reorthogonalization, sweep B (coefficients at small+coef):
//   q     <- cq * q - sum_k a_k V_k        (the reorthogonalized, normalized q)
//   qnext <- w - sum_k c_k V_k - cw * q_old (the next vector, projected once)
// with a = coef[0, nv), c = coef[nv, 2 nv), cq = coef[2 nv], cw = coef[2 nv + 1];
// chunk partial of qnext . qnext into part row 0.  One read of V, q, w.
__global__ __launch_bounds__(256) void k_update2_(const ProbDesc* __restrict__ probs,
                                                  const int2* __restrict__ work, int sbase, int nv, int sq,
                                                  int sw, int snext, int coef_off) {
  __shared__ double sh[4];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const LevelDesc& L = P.lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  const double* cf = P.small + coef_off;
  constexpr int NQ = TG_VCHUNK / 256;
  double ta[NQ], tc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) ta[q] = tc[q] = 0.0;
  // whole chunks (see k_dots2_); on the zero tail every value written is 0
  for (int k = 0; k < nv; ++k) {
    const double ak = cf[k], ck = cf[nv + k];
    const auto* v = gp(L.vec64 + (long long)(sbase + k) * L.stride);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double x = v[lo + threadIdx.x + 256LL * q];
      ta[q] += ak * x;
      tc[q] += ck * x;
    }
  }
  const double cq = cf[2 * nv], cw = cf[2 * nv + 1];
  auto* qv = gp(L.vec64 + (long long)sq * L.stride);
  const auto* wv = gp(L.vec64 + (long long)sw * L.stride);
  auto* nv_ = gp(L.vec64 + (long long)snext * L.stride);
  double nn = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const long long idx = lo + threadIdx.x + 256LL * q;
    const double qo = qv[idx];
    const double nx = wv[idx] - tc[q] - cw * qo;
    qv[idx] = cq * qo - ta[q];
    nv_[idx] = nx;
    nn += nx * nx;
  }
  nn = block_sum256(nn, sh);
  if (threadIdx.x == 0) P.part[wi.y] = nn;
}

// dst = src * small[scal + sc_index]
__global__ __launch_bounds__(256) void k_scale_(const ProbDesc* __restrict__ probs,
                                                const int2* __restrict__ work, int src, int dst,
                                                int sidx) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const LevelDesc& L = P.lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  const double a = P.small[sidx];
  const auto* s = gp(L.vec64 + (long long)src * L.stride);
  auto* d = gp(L.vec64 + (long long)dst * L.stride);
  for (long long q = lo + threadIdx.x; q < hi; q += 256) d[q] = s[q] * a;
}

// ---------------------------------------------------------------------------
// FGMRES scalar kernels: one thread per problem (work list {p, 0}).
__global__ void k_init_small_(const ProbDesc* __restrict__ probs, const int2* __restrict__ work,
                              int total) {
  const ProbDesc& P = probs[work[blockIdx.x].x];
  for (int q = threadIdx.x; q < total; q += blockDim.x) P.small[q] = 0.0;
}

// Cycle start: beta = ||r|| (tmp[0] holds r.r); history and stop tests.
__global__ void k_cycle_start_(const ProbDesc* __restrict__ probs, const int2* __restrict__ work,
                               SmallOffs o, int k, int cap, double tol, double* status_out) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  if (threadIdx.x != 0) return;
  double* S = P.small;
  double* sc = S + o.scal;
  const double beta = sqrt(S[o.tmp]);
  if (k == 0) {
    sc[SC_BNORM] = beta;
    S[o.hist] = (beta > 0.0) ? 1.0 : 0.0;
  }
  const double bnorm = sc[SC_BNORM];
  const double rel = bnorm > 0.0 ? beta / bnorm : 0.0;
  if (k > 0) S[o.hist + k] = rel;   // cycle-start true residual replaces the projection
  double st = TG_RUNNING;
  if (!isfinite(beta)) st = TG_NONFINITE;
  else if (rel <= tol) st = TG_PROJ_CONVERGED;
  else if (k >= cap) st = TG_MAXIT;
  sc[SC_BETA] = beta;
  sc[SC_STATUS] = st;
  sc[SC_ITERS] = k;
  sc[SC_JDONE] = 0;
  sc[SC_EST] = rel;
  sc[SC_INV] = beta > 0.0 ? 1.0 / beta : 0.0;
  sc[SC_RHO] = beta;   // delayed form: V_0 holds r itself, first-pass norm beta
  for (int q = 0; q <= o.mmax; ++q) S[o.g + q] = 0.0;
  S[o.g] = beta;
  status_out[wi.x] = st;
}

// Arnoldi column j: h (accumulated) and tmp[0] = ||w||^2 after projection,
// scal[SC_HN] <- ||w||; apply Givens rotations, new rotation, history, stop tests.
__global__ void k_arnoldi_(const ProbDesc* __restrict__ probs, const int2* __restrict__ work,
                           SmallOffs o, int j, int k, int cap, double tol, double brk,
                           double* status_out) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  if (threadIdx.x != 0) return;
  double* S = P.small;
  double* sc = S + o.scal;
  const int ldh = o.mmax + 1;
  double* Hc = S + o.H + (long long)ldh * j;
  const double hn = sqrt(S[o.tmp]);
  const double wn0 = sqrt(fmax(sc[SC_FLAG], 0.0));   // ||w|| before projection
  bool finite = isfinite(hn);
  for (int i = 0; i <= j; ++i) {
    Hc[i] = S[o.h + i];
    finite = finite && isfinite(Hc[i]);
  }
  Hc[j + 1] = hn;
  double st = TG_RUNNING;
  if (!finite) {
    st = TG_NONFINITE;
    sc[SC_STATUS] = st;
    status_out[wi.x] = st;
    return;   // column j unusable: jdone stays j
  }
  for (int i = 0; i < j; ++i) {
    const double c = S[o.cs + i], s = S[o.sn + i];
    const double t = c * Hc[i] + s * Hc[i + 1];
    Hc[i + 1] = -s * Hc[i] + c * Hc[i + 1];
    Hc[i] = t;
  }
  const double d = hypot(Hc[j], Hc[j + 1]);
  if (!(d > 0.0) || !isfinite(d)) {
    st = TG_NONFINITE;
    sc[SC_STATUS] = st;
    status_out[wi.x] = st;
    return;
  }
  const double c = Hc[j] / d, s = Hc[j + 1] / d;
  S[o.cs + j] = c;
  S[o.sn + j] = s;
  Hc[j] = d;
  Hc[j + 1] = 0.0;
  const double gj = S[o.g + j];
  S[o.g + j + 1] = -s * gj;
  S[o.g + j] = c * gj;
  const int kk = (int)sc[SC_ITERS] + 1;   // iterations so far live on the device (k: the host's count)
  (void)k;
  const double est = fabs(S[o.g + j + 1]) / sc[SC_BNORM];
  S[o.hist + kk] = est;
  sc[SC_EST] = est;
  sc[SC_ITERS] = kk;
  sc[SC_JDONE] = j + 1;
  sc[SC_HN] = hn;
  sc[SC_INV] = hn > 0.0 ? 1.0 / hn : 0.0;
  if (est <= tol) st = TG_PROJ_CONVERGED;
  else if (hn <= brk * wn0) st = TG_BREAKDOWN;
  else if (kk >= cap) st = TG_MAXIT;
  sc[SC_STATUS] = st;
  status_out[wi.x] = st;
}

// Delayed reorthogonalization, after sweep A of step j.  V_0..V_{j-1} hold
// the final orthonormal q_i, V_j the once-projected q~_j with first-pass norm
// rho = scal[SC_RHO]; tmp holds [Q^T q~ | Q^T w | q~.q~, q~.w, w.w] with
// w = K z_j, z_j = M^-1 (q~_j / rho).  With S = Q^T q~ / rho:
//   nu = sqrt(q~.q~ / rho^2 - |S|^2),  q_j = (q~_j / rho - Q S) / nu.
// Column j-1 of H becomes final: [h1 + rho S ; rho nu] (h1 = its first-pass
// coefficients), replacing the tentative column and rotation of step j-1.
// The first-pass coefficients of column j are h1 = [Q^T w ; q_j . w]; the
// coefficients of sweep B go to tmp (see k_update2_).
// LDS ordering between the lanes of the one wave that runs a scalar part
// (the wave is in lockstep; the fence keeps the compiler and the LDS queue
// from moving a lane's reads above another lane's writes)
#define TG_WAVE_SYNC()                                       \
  do {                                                       \
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");   \
    __builtin_amdgcn_wave_barrier();                         \
  } while (0)

__device__ void dcgs_a_wave(const ProbDesc& P, int p, const SmallOffs& o, int j, double* status_out) {
  // one wave: the column and the rotations are read in parallel and rotated
  // in LDS by lane 0 (a chain of register operations rather than of round
  // trips through memory)
  __shared__ double sH[TG_MAX_RESTART + 2], sC[TG_MAX_RESTART + 1], sS[TG_MAX_RESTART + 1];
  __shared__ int bad;
  const int2 wi = make_int2(p, 0);
  const int lane = threadIdx.x;
  double* S = P.small;
  double* sc = S + o.scal;
  if (sc[SC_STATUS] != TG_RUNNING) return;
  double* tmp = S + o.tmp;
  double* h1 = S + o.h;
  const int ldh = o.mmax + 1;
  const double rho = sc[SC_RHO];
  const double alpha = tmp[2 * j] / (rho * rho), qw = tmp[2 * j + 1] / rho, ww = tmp[2 * j + 2];
  double ss = 0.0, sz = 0.0;
  for (int k = lane; k < j; k += 64) {
    const double sk = tmp[k] / rho;
    ss += sk * sk;
    sz += sk * tmp[j + k];
  }
  ss = wave_sum(ss);
  sz = wave_sum(sz);
  const double nu2 = alpha - ss;
  double st = TG_RUNNING;
  if (!isfinite(nu2) || !isfinite(qw) || !isfinite(sz)) st = TG_NONFINITE;
  else if (!(nu2 > 0.0)) st = TG_BREAKDOWN;   // q~_j lies in span(Q): nothing new
  if (st != TG_RUNNING) {
    if (lane == 0) {
      sc[SC_STATUS] = st;
      status_out[wi.x] = st;
    }
    return;
  }
  const double nu = sqrt(nu2);
  if (lane == 0) sc[SC_FLAG] = ww;
  if (j >= 1) {
    double* Hc = S + o.H + (long long)ldh * (j - 1);
    for (int i = lane; i < j; i += 64) sH[i] = h1[i] + tmp[i];
    for (int i = lane; i < j - 1; i += 64) {
      sC[i] = S[o.cs + i];
      sS[i] = S[o.sn + i];
    }
    TG_WAVE_SYNC();
    if (lane == 0) {
      sH[j] = rho * nu;
      double carry = sH[0];
      for (int i = 0; i < j - 1; ++i) {
        const double c = sC[i], sn = sS[i], b = sH[i + 1];
        sH[i] = c * carry + sn * b;
        carry = -sn * carry + c * b;
      }
      sH[j - 1] = carry;
      const double d = hypot(sH[j - 1], sH[j]);
      bad = !(d > 0.0) || !isfinite(d);
      if (bad) {
        sc[SC_STATUS] = TG_NONFINITE;
        status_out[wi.x] = TG_NONFINITE;
      } else {
        const double c = sH[j - 1] / d, sn = sH[j] / d;
        S[o.cs + j - 1] = c;
        S[o.sn + j - 1] = sn;
        sH[j - 1] = d;
        sH[j] = 0.0;
        const double gj = sc[SC_GJ];
        S[o.g + j - 1] = c * gj;
        S[o.g + j] = -sn * gj;
      }
    }
    TG_WAVE_SYNC();
    for (int i = lane; i <= j; i += 64) Hc[i] = sH[i];
    if (bad) return;
  }
  const double hjj = (qw - sz) / nu;
  for (int k = lane; k < j; k += 64) {
    const double sk = tmp[k] / rho, zk = tmp[j + k];
    h1[k] = zk;
    tmp[j + k] = zk - sk * hjj / nu;
    tmp[k] = sk / nu;
  }
  if (lane == 0) {
    h1[j] = hjj;
    tmp[2 * j] = 1.0 / (rho * nu);
    tmp[2 * j + 1] = hjj / (nu * rho);
  }
}

// After sweep B of step j: rho' = ||q~_{j+1}|| (tmp[0]).  Column j enters
// tentatively as [h1 ; rho'] (its reorthogonalization correction is known
// only after the next sweep A): rotations, projected residual estimate,
// history and stop tests as in the immediate form.
__device__ void dcgs_b_wave(const ProbDesc& P, int p, const SmallOffs& o, int j, int cap, double tol, double brk,
                            double* status_out) {
  __shared__ double sH[TG_MAX_RESTART + 2], sC[TG_MAX_RESTART + 1], sS[TG_MAX_RESTART + 1];
  __shared__ int bad;
  const int2 wi = make_int2(p, 0);
  const int lane = threadIdx.x;
  double* S = P.small;
  double* sc = S + o.scal;
  if (sc[SC_STATUS] != TG_RUNNING) return;   // stopped in sweep A of this step
  const double* h1 = S + o.h;
  const int ldh = o.mmax + 1;
  const double rn = sqrt(S[o.tmp]);
  double* Hc = S + o.H + (long long)ldh * j;
  bool finite = true;
  for (int i = lane; i <= j; i += 64) {
    sH[i] = h1[i];
    finite = finite && isfinite(sH[i]);
  }
  for (int i = lane; i < j; i += 64) {
    sC[i] = S[o.cs + i];
    sS[i] = S[o.sn + i];
  }
  finite = __all(finite) && isfinite(rn);
  if (!finite) {
    for (int i = lane; i <= j; i += 64) Hc[i] = sH[i];
    if (lane == 0) {
      Hc[j + 1] = rn;
      sc[SC_STATUS] = TG_NONFINITE;
      status_out[wi.x] = TG_NONFINITE;
    }
    return;
  }
  TG_WAVE_SYNC();
  if (lane == 0) {
    sH[j + 1] = rn;
    double carry = sH[0];
    for (int i = 0; i < j; ++i) {
      const double c = sC[i], sn = sS[i], b = sH[i + 1];
      sH[i] = c * carry + sn * b;
      carry = -sn * carry + c * b;
    }
    sH[j] = carry;
    const double d = hypot(sH[j], sH[j + 1]);
    bad = !(d > 0.0) || !isfinite(d);
    if (bad) {
      sc[SC_STATUS] = TG_NONFINITE;
      status_out[wi.x] = TG_NONFINITE;
    } else {
      const double c = sH[j] / d, sn = sH[j + 1] / d;
      S[o.cs + j] = c;
      S[o.sn + j] = sn;
      sH[j] = d;
      sH[j + 1] = 0.0;
      const double gj = S[o.g + j];
      sc[SC_GJ] = gj;
      S[o.g + j + 1] = -sn * gj;
      S[o.g + j] = c * gj;
      const int kk = (int)sc[SC_ITERS] + 1;   // iterations so far live on the device
      const double est = fabs(S[o.g + j + 1]) / sc[SC_BNORM];
      S[o.hist + kk] = est;
      sc[SC_EST] = est;
      sc[SC_ITERS] = kk;
      sc[SC_JDONE] = j + 1;
      sc[SC_HN] = rn;
      sc[SC_RHO] = rn;
      sc[SC_INV] = rn > 0.0 ? 1.0 / rn : 0.0;
      double st = TG_RUNNING;
      if (est <= tol) st = TG_PROJ_CONVERGED;
      else if (rn <= brk * sqrt(fmax(sc[SC_FLAG], 0.0))) st = TG_BREAKDOWN;
      else if (kk >= cap) st = TG_MAXIT;
      sc[SC_STATUS] = st;
      status_out[wi.x] = st;
    }
  }
  TG_WAVE_SYNC();
  for (int i = lane; i <= j + 1; i += 64) Hc[i] = sH[i];
}

// The scalar ends of the two sweeps of a delayed-CGS2 step, one workgroup per
// problem: the chunk partials summed in a fixed order into small+tmp, then the
// step's scalar part on one wave.  A: rows [V.q | V.w | q.q, q.w, w.w], each
// summed over the chunks in chunk order; B: ||q_next||^2 over the chunks.
__global__ __launch_bounds__(256) void k_fin_a_(const ProbDesc* __restrict__ probs, const int2* __restrict__ work,
                                                SmallOffs o, int j, double* status_out) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const int nc = P.lv[0].n_chunks;
  double* tmp = P.small + o.tmp;
  for (int r = threadIdx.x; r < 2 * j + 3; r += 256) {
    const double* pr = P.part + (long long)r * nc;
    double a = 0.0;
#pragma unroll 8
    for (int c = 0; c < nc; ++c) a += pr[c];
    tmp[r] = a;
  }
  __syncthreads();
  if (threadIdx.x < 64) dcgs_a_wave(P, wi.x, o, j, status_out);
}
__global__ __launch_bounds__(256) void k_fin_b_(const ProbDesc* __restrict__ probs, const int2* __restrict__ work,
                                                SmallOffs o, int j, int cap, double tol, double brk,
                                                double* status_out) {
  __shared__ double sh[4];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const int nc = P.lv[0].n_chunks;
  double a = 0.0;
  for (int c = threadIdx.x; c < nc; c += 256) a += P.part[c];
  a = block_sum256(a, sh);
  if (threadIdx.x == 0) P.small[o.tmp] = a;
  __syncthreads();
  if (threadIdx.x < 64) dcgs_b_wave(P, wi.x, o, j, cap, tol, brk, status_out);
}

// Least squares: y = R^{-1} g over the jdone columns (back substitution).
__global__ void k_lsq_(const ProbDesc* __restrict__ probs, const int2* __restrict__ work, SmallOffs o) {
  const ProbDesc& P = probs[work[blockIdx.x].x];
  if (threadIdx.x != 0) return;
  double* S = P.small;
  const int jd = (int)S[o.scal + SC_JDONE];
  const int ldh = o.mmax + 1;
  for (int i = jd - 1; i >= 0; --i) {
    double v = S[o.g + i];
    for (int c = i + 1; c < jd; ++c) v -= S[o.H + (long long)ldh * c + i] * S[o.y + c];
    S[o.y + i] = v / S[o.H + (long long)ldh * i + i];
  }
  for (int i = jd; i < o.mmax; ++i) S[o.y + i] = 0.0;
}

// x += sum_{j < jdone} y_j Z_j
__global__ __launch_bounds__(256) void k_xupdate_(const ProbDesc* __restrict__ probs,
                                                  const int2* __restrict__ work, SmallOffs o,
                                                  int sz0) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  const LevelDesc& L = P.lv[0];
  long long lo, hi;
  chunk_range(L, wi.y, lo, hi);
  const int jd = (int)P.small[o.scal + SC_JDONE];
  auto* x = gp(L.vec64 + (long long)S_X * L.stride);
  double acc[TG_VCHUNK / 256];
#pragma unroll
  for (int q = 0; q < TG_VCHUNK / 256; ++q) acc[q] = 0.0;
  for (int jj = 0; jj < jd; ++jj) {
    const double yj = P.small[o.y + jj];
    const auto* z = gp(L.vec64 + (long long)(sz0 + jj) * L.stride);
#pragma unroll
    for (int q = 0; q < TG_VCHUNK / 256; ++q) {
      const long long idx = lo + threadIdx.x + 256LL * q;
      if (idx < hi) acc[q] += yj * z[idx];
    }
  }
#pragma unroll
  for (int q = 0; q < TG_VCHUNK / 256; ++q) {
    const long long idx = lo + threadIdx.x + 256LL * q;
    if (idx < hi) x[idx] += acc[q];
  }
}

// eta = sqrt(r.r / f.f) with tmp[0] = r.r, tmp[1] = f.f.  A zero right-hand
// side solved exactly (r.r = f.f = 0) gives 0; any other f.f that is not a
// finite positive number (a non-finite entry in f, or f.f = 0 with r != 0)
// gives NaN, which no acceptance test passes.
__global__ void k_true_eta_(const ProbDesc* __restrict__ probs, const int2* __restrict__ work,
                            SmallOffs o, double* out) {
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  if (threadIdx.x != 0) return;
  const double rr = P.small[o.tmp], ff = P.small[o.tmp + 1];
  double eta;
  if (rr == 0.0 && ff == 0.0)
    eta = 0.0;
  else if (ff > 0.0 && isfinite(ff))
    eta = sqrt(rr / ff);   // NaN when r.r is NaN, +inf when it overflows
  else
    eta = __builtin_nan("");
  P.small[o.scal + SC_TRUE] = eta;
  if (out) out[wi.x] = eta;
}

// ===========================================================================
// Launch wrappers.  Each launch of a timed class is bracketed by timer events
// (when the timer is on) and charged its algorithmic HBM bytes.
static inline dim3 nblk(const DevList& d) { return dim3((unsigned)d.n); }

static SmallOffs offs(const Batch* b) {
  const SmallLayout& s = b->grids[0]->sl;
  SmallOffs o;
  o.mmax = s.mmax;
  o.H = s.H;
  o.g = s.g;
  o.cs = s.cs;
  o.sn = s.sn;
  o.y = s.y;
  o.h = s.h;
  o.tmp = s.tmp;
  o.scal = s.scal;
  o.hist = s.hist;
  return o;
}

static int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  return TG_OK;
}

// Sums over the active problems that take part in a level-l launch.
// mode 0: every problem with level l; 1: l is not its coarsest; 2: l is its coarsest
static void level_sums(const Batch* b, int l, int mode, double& nodes, double& elems, double& cdof2) {
  nodes = elems = cdof2 = 0;
  for (int p : b->active) {
    const tg_grid* g = b->grids[p];
    if (l >= g->nlev) continue;
    if (mode == 1 && l == g->nlev - 1) continue;
    if (mode == 2 && l != g->nlev - 1) continue;
    nodes += (double)g->lv[l].n_nodes;
    elems += (double)g->lv[l].n_elem;
    cdof2 += (double)g->ncoarse * g->ncoarse;
  }
}
static double dofs0(const Batch* b) {
  double n = 0;
  for (int p : b->active) n += 3.0 * b->grids[p]->lv[0].n_nodes;
  return n;
}

#define TG_TIMED(kind, bytes_expr, ...)                 \
  do {                                                  \
    void* _th = timer_begin((kind), s);                 \
    __VA_ARGS__;                                        \
    if (_th) timer_end(_th, (double)(bytes_expr), s);   \
  } while (0)

// Largest coarsest level (free DOFs) whose two packed triangles fit the
// dynamic LDS the set-up kernel may take on the current device (the
// device's per-workgroup limit less the kernel's static LDS), with the
// kernel's limit raised to it once per device.
static size_t coarse_lds_limit();
// LDS doubles k_coarse_factor_lds needs for a coarsest level of n free
// DOFs: the assembled matrix and two pivot rows (LDS form), or the two pivot
// buffers of the register form when it applies.
static size_t coarse_lds_words(int n) {
  size_t w = (size_t)n * (n + 2);
  const int rpp = CF_THREADS / n, cm = (n + rpp - 1) / rpp;
  if (n >= 2 && cm <= CF_REG) w = std::max(w, (size_t)2 * (rpp * cm + CF_REG + n));
  return w;
}
static int coarse_lds_n() {
  const size_t lim = coarse_lds_limit();
  int n = 0;
  while (sizeof(double) * (size_t)(n + 1) * (n + 3) <= lim) ++n;   // (n + 1)^2 + 2 (n + 1)
  return n;
}
static size_t coarse_lds_limit() {
  static size_t lim[64] = {};
  static bool done[64] = {};
  static std::mutex mu;   // batches on several host threads
  std::lock_guard<std::mutex> lk(mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (!done[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
      (void)hipGetLastError();   // leave no error for the next launch check
      v = 0;
    }
    size_t l = v > 1024 ? (size_t)v - 1024 : 0;
    if (l && hipFuncSetAttribute((const void*)k_coarse_factor_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)l) != hipSuccess) {
      (void)hipGetLastError();
      l = std::min<size_t>(l, 65536 - 1024);
    }
    lim[dev] = l;
    done[dev] = true;
  }
  return lim[dev];
}

int k_set_density(Batch* b, hipStream_t s) {
  int* bad = b->flag_d;
  TG_HIP(hipMemsetAsync(bad, 0, sizeof(int) * b->n, s));
  TG_TIMED(TG_KT_SETUP, 0, {
    if (b->elem[0].n) k_young<<<nblk(b->elem[0]), 256, 0, s>>>(b->desc_d, b->elem[0].ptr, b->p, bad);
    if (b->elem[1].n) k_galerkin1<<<nblk(b->elem[1]), 256, 0, s>>>(b->desc_d, b->elem[1].ptr);
    for (int l = 2; l < b->maxlev; ++l)
      if (b->elem[l].n) k_galerkin_up<<<nblk(b->elem[l]), 256, 0, s>>>(b->desc_d, b->elem[l].ptr, l);
    for (int l = TG_MF_LEVELS + 1; l < b->maxlev; ++l)
      if (b->elem[l].n) k_mode_pack<<<nblk(b->elem[l]), 256, 0, s>>>(b->desc_d, b->elem[l].ptr, l);
    for (int l = 0; l < b->maxlev; ++l)
      if (b->node[l].n) k_nodeblock<<<nblk(b->node[l]), 256, 0, s>>>(b->desc_d, b->node[l].ptr, l);
    if (b->prob.n) {
      // which kernel sets up a problem depends only on its own coarsest size
      // and the device, so a problem gets the same inverse alone or batched
      const int nlds = coarse_lds_n();
      int nmax = 0, nmin = INT_MAX;
      for (int p : b->active) {
        const int n = b->grids[p]->ncoarse;
        if (n > 0) nmax = std::max(nmax, n), nmin = std::min(nmin, n);
      }
      if (nmin <= nlds) {
        size_t words = 0;
        for (int p : b->active) {
          const int n = b->grids[p]->ncoarse;
          if (n > 0 && n <= nlds) words = std::max(words, coarse_lds_words(n));
        }
        k_coarse_factor_lds<<<nblk(b->prob), CF_THREADS, sizeof(double) * words, s>>>(b->desc_d, b->prob.ptr,
                                                                                        bad, nlds);
      }
      if (nmax > nlds) k_coarse_factor<<<nblk(b->prob), 256, 0, s>>>(b->desc_d, b->prob.ptr, bad, nlds + 1);
    }
  });
  return check_launch("set_density kernels");
}

// fine-level operator of type T on list dl (mode: 0 apply, 1 resid, 2 smooth)
template <class T>
static double op_bytes(const Batch* b, int l, int lmode, int op) {
  double nodes, elems, c2;
  level_sums(b, l, lmode, nodes, elems, c2);
  const double vec = 3.0 * nodes * sizeof(T);
  // fine level and matrix-free Galerkin levels read the fine moduli; deeper
  // levels read their stored mode-basis element matrices
  const double mat = (l <= TG_MF_LEVELS) ? elems * double(1 << (3 * l)) * sizeof(T) : elems * double(TG_GM_NU) * sizeof(T);
  const double dinv = (op == OP_SMOOTH) ? 9.0 * nodes * sizeof(T) : 0.0;
  const int nvec = op == OP_APPLY ? 2 : 3;
  // the fused restriction reads x and b and writes the coarse right-hand side
  if (op == OP_RESTRICT) return 2 * vec + mat + vec / 8.0;
  // the fused first sweeps read b in FP64 and the node blocks, write x and b's copy
  if (op == OP_SMOOTH1) return 3.0 * nodes * 8.0 + 9.0 * nodes * sizeof(T) + mat + 2 * vec;
  return nvec * vec + mat + dinv;
}

int k_apply(Batch* b, int prec, int sx, const void* ex, int sy, void* ey, hipStream_t s) {
  if (prec == TG_BF16MFMA || prec == TG_BF16X3MFMA)
    TG_TIMED(TG_KT_VCYCLE_FINE, (op_bytes<float>(b, 0, 0, OP_APPLY)),
             launch_fine_mfma(b, b->fine, OP_APPLY, prec == TG_BF16X3MFMA, sx, ex, 0, nullptr, sy, ey, 0.0,
                              false, s));
  else if (prec == TG_F64)
    TG_TIMED(TG_KT_APPLY_F64, (op_bytes<double>(b, 0, 0, OP_APPLY)),
             launch_fine<double>(b, b->fine, 0, OP_APPLY, sx, ex, 0, nullptr, sy, ey, 0.0, s));
  else
    TG_TIMED(TG_KT_VCYCLE_FINE, (op_bytes<float>(b, 0, 0, OP_APPLY)),
             launch_fine<float>(b, b->fine, 0, OP_APPLY, sx, ex, 0, nullptr, sy, ey, 0.0, s));
  return check_launch("apply_K");
}

int k_residual64(Batch* b, int sb, int sx, int sy, hipStream_t s) {
  TG_TIMED(TG_KT_APPLY_F64, (op_bytes<double>(b, 0, 0, OP_RESID)),
           launch_fine<double>(b, b->fine, 0, OP_RESID, sx, nullptr, sb, nullptr, sy, nullptr, 0.0, s));
  return check_launch("residual");
}

// mf: 0 = vector mode-basis contraction, 1 = BF16 matrix cores, 2 = split BF16
template <class T, int OP>
// (y: slot of level l, or for OP_RESTRICT the right-hand-side slot of level
// l + 1, with y2 that level's first-sweep slot)
static void vc_op(Batch* b, int l, int x, int bs, int y, T om, hipStream_t s, int mf = 0, int y2 = -1,
                  int vbs = 0) {
  const DevList& dl = (OP == OP_RESTRICT) ? b->zm_r[l] : b->zm_s[l];
  if (l == 0 && mf)
    TG_TIMED(TG_KT_VCYCLE_FINE, (op_bytes<T>(b, 0, 1, OP)),
             launch_fine_mfma(b, dl, OP, mf == 2, x, nullptr, bs, nullptr, y, nullptr, (double)om, false, s, y2));
  else if (l == 0)
    TG_TIMED(TG_KT_VCYCLE_FINE, (op_bytes<T>(b, 0, 1, OP)),
             launch_fine<T>(b, dl, 0, OP, x, nullptr, bs, nullptr, y, nullptr, (double)om, s, y2));
  else
    TG_TIMED(TG_KT_VCYCLE_COARSE, (op_bytes<T>(b, l, 1, OP)),
             launch_fine<T>(b, dl, l, OP, x, nullptr, bs, nullptr, y, nullptr, (double)om, s, y2, vbs));
}

// One fixed V-cycle.  Level-0 input b (slot sb of the FP64 pool or external
// eb, typed double unless in_is_f32) -> output (slot sy of the FP64 pool or
// external ey, double unless out_is_f32).
template <class T>
static int vcycle_t(Batch* b, int in_is_f32, int sb, const void* eb, int out_is_f32, int sy,
                    void* ey, hipStream_t s, int mf, int in_scale) {
  const tg_mg_opts& mg = b->grids[0]->mg;
  const T om = T(mg.omega);
  const bool f64 = sizeof(T) == 8;
  const int B0 = f64 ? S_VB : C_B, XA0 = f64 ? S_VXA : C_XA, XB0 = f64 ? S_VXB : C_XB;
  const int flips = (mg.nu_pre - 1) + mg.nu_post;
  const int FIN = (flips % 2 == 0) ? C_XA : C_XB;      // level >= 1 result slot
  const int FIN0 = (flips % 2 == 0) ? XA0 : XB0;
  int cur[TG_MAXLEV];
  const int L = b->maxlev;
  double nodes, elems, c2;
  const double sT = sizeof(T), sIn = in_is_f32 ? 4.0 : 8.0, sOut = out_is_f32 ? 4.0 : 8.0;
  // Fast level-0 boundary: FGMRES calls with an FP64 slot in, an FP64 slot out
  // and every problem multilevel.  The first sweep reads the FP64 vector
  // directly and the last sweep writes the FP64 output.
  bool all_multi = true;
  for (int p : b->active) all_multi = all_multi && b->grids[p]->nlev > 1;
  const bool fast_in = !in_is_f32 && sb >= 0 && all_multi;
  const bool fast_out = !out_is_f32 && sy >= 0 && all_multi;
  // The bottom of the cycle (each problem's levels from its vb_lb down) runs
  // as one launch between the two passes; the level-by-level launches skip
  // those levels (vbs) and whole levels no problem needs.
  const int tv = f64 ? 1 : 0;
  const bool use_vb = b->vb[tv].n > 0;
  const int vbs = use_vb ? 1 : 0;
  auto level_needed = [&](int l) { return !use_vb || b->vb_need[tv][l]; };
  // ---- descend
  for (int l = 0; l < L; ++l) {
    if (!level_needed(l)) continue;
    const int Bs = l == 0 ? B0 : C_B, XA = l == 0 ? XA0 : C_XA, XB = l == 0 ? XB0 : C_XB;
    const DevList& sm = b->smooth[l];
    const DevList& co = b->coarse[l];
    if (l == 0 && b->node[0].n && !fast_in) {
      // b into the working slot of type T (also masks the clamped nodes)
      level_sums(b, 0, 0, nodes, elems, c2);
      if (in_is_f32)
        TG_TIMED(TG_KT_TRANSFER, 3.0 * nodes * (sIn + sT),
                 k_copy_level<float, T><<<nblk(b->node[0]), 256, 0, s>>>(b->desc_d, b->node[0].ptr, 0, sb, eb, Bs, nullptr, in_scale));
      else
        TG_TIMED(TG_KT_TRANSFER, 3.0 * nodes * (sIn + sT),
                 k_copy_level<double, T><<<nblk(b->node[0]), 256, 0, s>>>(b->desc_d, b->node[0].ptr, 0, sb, eb, Bs, nullptr, in_scale));
    }
    if (co.n) {
      const int fin = l == 0 ? FIN0 : FIN;
      level_sums(b, l, 2, nodes, elems, c2);
      TG_TIMED(TG_KT_TRANSFER, c2 * sT + 6.0 * nodes * sT,
               k_coarse_solve<T, T, T><<<nblk(co), 256, 0, s>>>(b->desc_d, co.ptr, l, Bs, nullptr, fin, nullptr,
                                                                vbs));
    }
    if (!sm.n) continue;
    level_sums(b, l, 1, nodes, elems, c2);
    int c = XA, o = XB;
    int it0 = 1;
    if (l == 0 && fast_in && mg.nu_pre >= 2) {
      // first sweep from zero computed while staging, second sweep in the same pass
      vc_op<T, OP_SMOOTH1>(b, 0, in_scale, sb, o, om, s, mf, Bs, vbs);
      std::swap(c, o);
      it0 = 2;
    } else if (l == 0 && fast_in)
      TG_TIMED(TG_KT_TRANSFER, 3.0 * nodes * (8.0 + 2 * sT) + 9.0 * nodes * sT,
               k_jacobi_first<double, T><<<nblk(sm), 256, 0, s>>>(b->desc_d, sm.ptr, 0, sb, nullptr, Bs, XA, om,
                                                                    in_scale));
    else if (l == 0)
      TG_TIMED(TG_KT_TRANSFER, 3.0 * nodes * 2 * sT + 9.0 * nodes * sT,
               k_jacobi_first<T, T><<<nblk(sm), 256, 0, s>>>(b->desc_d, sm.ptr, l, Bs, nullptr, INT_MIN, XA, om, -1));
    // (levels >= 1: the restriction above already wrote the first sweep)
    for (int it = it0; it < mg.nu_pre; ++it) {
      vc_op<T, OP_SMOOTH>(b, l, c, Bs, o, om, s, mf, -1, vbs);
      std::swap(c, o);
    }
    // residual, restricted straight into the next level's right-hand side,
    // and that level's first Jacobi sweep from zero
    vc_op<T, OP_RESTRICT>(b, l, c, Bs, C_B, om, s, mf, C_XA, vbs);
    cur[l] = c;
  }
  if (use_vb)
    TG_TIMED(TG_KT_VCYCLE_COARSE, vbottom_bytes(b, tv),
             launch_vbottom<T>(b, b->vb[tv], b->vb_lds[tv], FIN, mg.omega, mg.nu_pre, mg.nu_post, b->vb_l1[tv], s));
  // ---- ascend
  for (int l = L - 1; l >= 0; --l) {
    const DevList& sm = b->smooth[l];
    if (!sm.n || !level_needed(l)) continue;
    const int Bs = l == 0 ? B0 : C_B, XA = l == 0 ? XA0 : C_XA, XB = l == 0 ? XB0 : C_XB;
    int c = cur[l];
    int o = (c == XA) ? XB : XA;
    level_sums(b, l, 1, nodes, elems, c2);
    TG_TIMED(TG_KT_TRANSFER, 3.0 * nodes * 2 * sT + 3.0 * nodes / 8 * sT,
             k_prolong<T><<<nblk(sm), 256, 0, s>>>(b->desc_d, sm.ptr, l, c, FIN, nullptr, nullptr, vbs));
    for (int it = 0; it < mg.nu_post; ++it) {
      if (l == 0 && fast_out && it == mg.nu_post - 1) {
        if (f64)
          vc_op<T, OP_SMOOTH>(b, 0, c, Bs, sy, om, s, 0, -1, vbs);   // straight into the FP64 output slot
        else if (mf)
          TG_TIMED(TG_KT_VCYCLE_FINE, (op_bytes<T>(b, 0, 1, OP_SMOOTH) + 3.0 * nodes * (8.0 - sT)),
                   launch_fine_mfma(b, b->zm_s[0], OP_SMOOTH, mf == 2, c, nullptr, Bs, nullptr, sy, nullptr,
                                    (double)om, true, s));
        else
          TG_TIMED(TG_KT_VCYCLE_FINE, (op_bytes<T>(b, 0, 1, OP_SMOOTH) + 3.0 * nodes * (8.0 - sT)),
                   launch_fine_smooth_out64(b, b->zm_s[0], c, Bs, sy, (double)om, s));
        c = -1;   // result is in the output slot
        break;
      }
      vc_op<T, OP_SMOOTH>(b, l, c, Bs, o, om, s, mf, -1, vbs);
      std::swap(c, o);
    }
    cur[l] = c;
  }
  // ---- output (level 0): result in FIN0 for every problem
  if (b->node[0].n && !fast_out) {
    level_sums(b, 0, 0, nodes, elems, c2);
    if (out_is_f32)
      TG_TIMED(TG_KT_TRANSFER, 3.0 * nodes * (sOut + sT),
               k_copy_level<T, float><<<nblk(b->node[0]), 256, 0, s>>>(b->desc_d, b->node[0].ptr, 0, FIN0, nullptr, sy, ey, -1));
    else
      TG_TIMED(TG_KT_TRANSFER, 3.0 * nodes * (sOut + sT),
               k_copy_level<T, double><<<nblk(b->node[0]), 256, 0, s>>>(b->desc_d, b->node[0].ptr, 0, FIN0, nullptr, sy, ey, -1));
  }
  return check_launch("vcycle");
}

int k_vcycle(Batch* b, int prec, int in_is_f32, int sb, const void* eb, int out_is_f32, int sy,
             void* ey, hipStream_t s, int in_scale_sc) {
  const int in_scale = in_scale_sc >= 0 ? offs(b).scal + in_scale_sc : -1;
  if (prec == TG_F64) return vcycle_t<double>(b, in_is_f32, sb, eb, out_is_f32, sy, ey, s, 0, in_scale);
  const int mf = prec == TG_BF16MFMA ? 1 : prec == TG_BF16X3MFMA ? 2 : 0;
  return vcycle_t<float>(b, in_is_f32, sb, eb, out_is_f32, sy, ey, s, mf, in_scale);
}

// ---- level primitives of host-stepped cycles (FP64, external vectors of
// the level's full length, clamped nodes zero)
int level_op64(Batch* b, int l, int op, const double* x, const double* bb, double* y, double omega,
               hipStream_t s) {
  const bool all = (l == 0 && op == OP_APPLY);
  const DevList& dl = all ? b->fine : b->zm_s[l];
  TG_TIMED(l == 0 ? TG_KT_APPLY_F64 : TG_KT_VCYCLE_COARSE, (op_bytes<double>(b, l, all ? 0 : 1, op)),
           launch_fine<double>(b, dl, l, op, -1, x, -1, bb, -1, y, omega, s));
  return check_launch("level operator");
}
int level_restrict64(Batch* b, int l, const double* x, const double* bb, int slot_next, hipStream_t s) {
  TG_TIMED(l == 0 ? TG_KT_APPLY_F64 : TG_KT_VCYCLE_COARSE, (op_bytes<double>(b, l, 1, OP_RESTRICT)),
           launch_fine<double>(b, b->zm_r[l], l, OP_RESTRICT, -1, x, -1, bb, slot_next, nullptr, 0.0, s, -1));
  return check_launch("level restriction");
}
int level_prolong64(Batch* b, int l, const double* ec, double* xf, hipStream_t s) {
  const DevList& sm = b->smooth[l];
  if (sm.n) {
    double nodes, elems, c2;
    level_sums(b, l, 1, nodes, elems, c2);
    TG_TIMED(TG_KT_TRANSFER, 3.0 * nodes * 16.0 + 3.0 * nodes / 8 * 8.0,
             k_prolong<double><<<nblk(sm), 256, 0, s>>>(b->desc_d, sm.ptr, l, -1, -1, ec, xf, 0));
  }
  return check_launch("level prolongation");
}
int level_coarse64(Batch* b, int l, const double* bb, double* y, hipStream_t s) {
  const DevList& co = b->coarse[l];
  if (co.n) {
    double nodes, elems, c2;
    level_sums(b, l, 2, nodes, elems, c2);
    TG_TIMED(TG_KT_TRANSFER, c2 * 8.0 + 6.0 * nodes * 8.0,
             k_coarse_solve<double, double, double><<<nblk(co), 256, 0, s>>>(b->desc_d, co.ptr, l, -1, bb, -1, y,
                                                                             0));
  }
  return check_launch("coarsest solve");
}

int k_copy_ext(Batch* b, int dir, int slot, hipStream_t s) {
  if (b->vec.n)
    TG_TIMED(TG_KT_UPDATE, 16.0 * dofs0(b), k_copy_ext_<<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, dir, slot));
  return check_launch("copy_ext");
}
int k_fill0(Batch* b, int slot, double v, hipStream_t s) {
  if (b->vec.n)
    TG_TIMED(TG_KT_UPDATE, 8.0 * dofs0(b), k_fill0_<<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, slot, v));
  return check_launch("fill");
}
int k_copy0(Batch* b, int src, int dst, hipStream_t s) {
  if (b->vec.n)
    TG_TIMED(TG_KT_UPDATE, 16.0 * dofs0(b), k_copy0_<<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, src, dst));
  return check_launch("copy");
}
int k_multidot(Batch* b, int sbase, int nv, int sw, int with_self, hipStream_t s) {
  if (b->vec.n)
    TG_TIMED(TG_KT_MULTIDOT, 8.0 * (nv + 1) * dofs0(b),
             k_multidot_<<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, sbase, nv, sw, with_self));
  return check_launch("multidot");
}
int k_reduce(Batch* b, int nv, int mode, int dst, int save_k, hipStream_t s) {
  const SmallOffs o = offs(b);
  if (b->prob.n && nv > 0)
    TG_TIMED(TG_KT_SCALAR, 0,
             k_reduce_<<<dim3(b->prob.n, nv), 256, 0, s>>>(b->desc_d, b->prob.ptr, o.h, o.tmp + dst,
                                                          o.scal + SC_FLAG, mode, save_k));
  return check_launch("reduce");
}
int k_update(Batch* b, int sbase, int nv, int sw, int coef_is_tmp, hipStream_t s) {
  const SmallOffs o = offs(b);
  const int coef_off = coef_is_tmp ? o.tmp : o.h;
  if (b->vec.n)
    TG_TIMED(TG_KT_UPDATE, 8.0 * (nv + 2) * dofs0(b),
             k_update_<<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, sbase, nv, sw, coef_off));
  return check_launch("update");
}
int k_update_dots(Batch* b, int sbase, int nv, int sw, int coef_is_tmp, int ndot, int with_self,
                  hipStream_t s) {
  const SmallOffs o = offs(b);
  const int coef_off = coef_is_tmp ? o.tmp : o.h;
  if (b->vec.n) {
    if (nv <= 32 && ndot <= 32)
      TG_TIMED(TG_KT_UPDATE, 8.0 * (nv + 2) * dofs0(b),
               k_update_dots_reg_<32><<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, sbase, nv, sw,
                                                                  coef_off, ndot, with_self));
    else
      TG_TIMED(TG_KT_UPDATE, 8.0 * (nv + 2 + ndot) * dofs0(b),
               k_update_dots_<<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, sbase, nv, sw, coef_off,
                                                          ndot, with_self));
  }
  return check_launch("update_dots");
}

// Sweep A of the delayed CGS2 step j (nv = j basis vectors), then its
// scalar end (chunk sums and the first scalar part) in one per-problem launch.
int k_dots2(Batch* b, int sbase, int nv, int sq, int sw, hipStream_t s) {
  if (b->vec.n)
    TG_TIMED(TG_KT_MULTIDOT, 8.0 * (nv + 2) * dofs0(b),
             k_dots2_<<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, sbase, nv, sq, sw));
  if (b->prob.n)
    TG_TIMED(TG_KT_SCALAR, 0, k_fin_a_<<<nblk(b->prob), 256, 0, s>>>(b->desc_d, b->prob.ptr, offs(b), nv, b->sc_d));
  return check_launch("dots2");
}
// Sweep B, then its scalar end (the norm sum, the Givens update, the history
// entry and the stop tests) in one per-problem launch.
int k_update2(Batch* b, int sbase, int nv, int sq, int sw, int snext, int cap, double tol, double brk,
              hipStream_t s) {
  const SmallOffs o = offs(b);
  if (b->vec.n)
    TG_TIMED(TG_KT_UPDATE, 8.0 * (nv + 4) * dofs0(b),
             k_update2_<<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, sbase, nv, sq, sw, snext, o.tmp));
  if (b->prob.n)
    TG_TIMED(TG_KT_SCALAR, 0,
             k_fin_b_<<<nblk(b->prob), 256, 0, s>>>(b->desc_d, b->prob.ptr, o, nv, cap, tol, brk, b->sc_d));
  return check_launch("update2");
}
int k_scale_to(Batch* b, int src, int dst, int sc_index, hipStream_t s) {
  const int sidx = offs(b).scal + sc_index;
  if (b->vec.n)
    TG_TIMED(TG_KT_UPDATE, 16.0 * dofs0(b), k_scale_<<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, src, dst, sidx));
  return check_launch("scale");
}
int k_cycle_start(Batch* b, int k, int cap, double tol, hipStream_t s) {
  if (b->prob.n)
    TG_TIMED(TG_KT_SCALAR, 0,
             k_cycle_start_<<<nblk(b->prob), 64, 0, s>>>(b->desc_d, b->prob.ptr, offs(b), k, cap, tol, b->sc_d));
  return check_launch("cycle_start");
}
int k_arnoldi(Batch* b, int j, int k, int cap, double tol, double brk, hipStream_t s) {
  if (b->prob.n)
    TG_TIMED(TG_KT_SCALAR, 0,
             k_arnoldi_<<<nblk(b->prob), 64, 0, s>>>(b->desc_d, b->prob.ptr, offs(b), j, k, cap, tol, brk, b->sc_d));
  return check_launch("arnoldi");
}
int k_lsq_update(Batch* b, int mmax, int jmax, hipStream_t s) {
  const SmallOffs o = offs(b);
  if (b->prob.n) TG_TIMED(TG_KT_SCALAR, 0, k_lsq_<<<nblk(b->prob), 64, 0, s>>>(b->desc_d, b->prob.ptr, o));
  if (b->vec.n)
    TG_TIMED(TG_KT_UPDATE, 8.0 * (jmax + 2) * dofs0(b),
             k_xupdate_<<<nblk(b->vec), 256, 0, s>>>(b->desc_d, b->vec.ptr, o, slot_Z(mmax, 0)));
  return check_launch("lsq_update");
}
int k_true_eta(Batch* b, hipStream_t s, bool to_status) {
  if (b->prob.n)
    TG_TIMED(TG_KT_SCALAR, 0, k_true_eta_<<<nblk(b->prob), 64, 0, s>>>(b->desc_d, b->prob.ptr, offs(b),
                                                                        to_status ? b->sc_d : nullptr));
  return check_launch("true_eta");
}
int k_init_small(Batch* b, hipStream_t s) {
  if (b->prob.n)
    TG_TIMED(TG_KT_SCALAR, 0,
             k_init_small_<<<nblk(b->prob), 256, 0, s>>>(b->desc_d, b->prob.ptr, b->grids[0]->sl.total));
  return check_launch("init_small");
}

}  // namespace tg
