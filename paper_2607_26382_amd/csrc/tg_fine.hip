// Fine-level operator kernels: z-marching element columns, mode-basis Ke.
//
// A workgroup of 16x16 threads owns a 16x16 patch of element columns
// (ex, ey) = (x0 - 1 + tx, y0 - 1 + ty) and marches over element layers k.
// Thread (tx, ty) loads node (ex + 1, ey + 1) of every node layer; the other
// three top-face nodes of its element come from LDS.  Each element's 24
// outputs are formed in the polynomial-mode basis of the trilinear hex
// (per component: modes 1, x, y, xy, z, xz, yz, xyz), where Ke of a cube has
// 45 nonzeros (normal 3x3 block, rank-1 shear pairs, bilinear pairs and a
// triple, trilinear diagonal): ~205 flops instead of 1152 for the dense 24x24.
// The bottom-face outputs of layer k and the top-face outputs of layer k-1 are
// summed in registers, staged in LDS, and node (ex + 1, ey + 1) gathers its
// four in-plane element contributions: a complete, atomic-free, deterministic
// K u at node layer k, fused with the residual or the damped node-block Jacobi
// update.  Output nodes: 15 x 15 columns per workgroup, ZC node layers.
#include <cmath>
#include <mutex>
#include <cstring>
#include <vector>

#include "tg_internal.h"

// No implicit multiply-add contraction in this file: the z-march is unrolled,
// and the compiler could otherwise fuse a*b + c*d differently in the copies,
// making results depend on where a tile starts.  Fused operations are written
// out with mad_.
#pragma clang fp contract(off)

namespace tg {

__host__ __device__ __forceinline__ float mad_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double mad_(double a, double b, double c) { return __builtin_fma(a, b, c); }

enum { FOP_APPLY = 0, FOP_RESID = 1, FOP_SMOOTH = 2, FOP_RESTRICT = 3, FOP_SMOOTH1 = 4 };
// FOP_SMOOTH1 (level 0): the first two sweeps from x = 0 in one pass.  The
// right-hand side is read from an FP64 slot (sb), times the per-problem scale
// small[sx] when sx >= 0; every staged node gets x = w D^-1 b on the fly (the
// first sweep), the output is the second sweep x + w D^-1 (b - K x), and the
// FP32 copy of b that later sweeps read goes to slot sy2.

// Tiling of the residual sweep fused with the restriction (OP = FOP_RESTRICT):
// a tile owns 7 x 7 coarse node columns and m coarse node layers, and computes
// the fine residual on the 15 x 15 fine node columns and 2 m + 1 fine layers
// their 27-point stencils cover (fine columns 14 t - 1 .. 14 t + 13, layers
// 2 m t_z - 1 .. 2 m t_z + 2 m - 1).  Neighbouring tiles recompute one shared
// fine column / layer, so every coarse node is summed by one thread in one
// fixed order.
#define RZ_C 7
__host__ __device__ __forceinline__ int rz_layers(int zc) { return zc > 1 ? (zc + 1) / 2 : 1; }

// In-place 8-point transform along the three node-index bits:
// forward: (v0, v1) -> (v0 + v1, v1 - v0); node index a -> mode index m.
template <class T>
__device__ __forceinline__ void wht_fwd(T* v) {
#pragma unroll
  for (int b = 1; b < 8; b <<= 1)
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (!(a & b)) {
        const T x0 = v[a], x1 = v[a | b];
        v[a] = x0 + x1;
        v[a | b] = x1 - x0;
      }
}
// transpose transform: (b0, b1) -> (b0 - b1, b0 + b1); mode index -> node index
template <class T>
__device__ __forceinline__ void wht_inv(T* v) {
#pragma unroll
  for (int b = 1; b < 8; b <<= 1)
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (!(a & b)) {
        const T x0 = v[a], x1 = v[a | b];
        v[a] = x0 - x1;
        v[a | b] = x0 + x1;
      }
}

// The x and y stages of wht_fwd / wht_inv on one z-face (corner c = di + 2 dj).
// A face shared by two element layers is transformed once: the top face of
// layer k is the bottom face of layer k + 1, and the two layers' outputs on
// it are summed before its inverse stages.
template <class T>
__device__ __forceinline__ void face_fwd(T* v) {
#pragma unroll
  for (int b = 1; b < 4; b <<= 1)
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (!(a & b)) {
        const T x0 = v[a], x1 = v[a | b];
        v[a] = x0 + x1;
        v[a | b] = x1 - x0;
      }
}
template <class T>
__device__ __forceinline__ void face_inv(T* v) {
#pragma unroll
  for (int b = 1; b < 4; b <<= 1)
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (!(a & b)) {
        const T x0 = v[a], x1 = v[a | b];
        v[a] = x0 - x1;
        v[a | b] = x0 + x1;
      }
}

// mode_contract with the element modulus folded into the coefficients:
// c = (d - o, o, s, p, q, r - t, t, w) already multiplied by E.
template <class T>
struct ModeCoefE {
  T dmo, o, s, p, q, rmt, t, w;
};
template <class T>
__device__ __forceinline__ ModeCoefE<T> coef_times(const ModeCoefE<T>& c, T E) {
  return {c.dmo * E, c.o * E, c.s * E, c.p * E, c.q * E, c.rmt * E, c.t * E, c.w * E};
}
template <class T>
__device__ __forceinline__ void mode_contract_e(T* ux, T* uy, T* uz, const ModeCoefE<T>& c) {
  const T ns = ux[1] + uy[2] + uz[4];
  const T ons = c.o * ns;
  const T bxx = mad_(c.dmo, ux[1], ons), byy = mad_(c.dmo, uy[2], ons), bzz = mad_(c.dmo, uz[4], ons);
  const T sxy = c.s * (uy[1] + ux[2]);
  const T sxz = c.s * (uz[1] + ux[4]);
  const T syz = c.s * (uz[2] + uy[4]);
  const T p1a = mad_(c.p, ux[3], c.q * uz[6]), p1b = mad_(c.q, ux[3], c.p * uz[6]);
  const T p2a = mad_(c.p, uy[3], c.q * uz[5]), p2b = mad_(c.q, uy[3], c.p * uz[5]);
  const T p3a = mad_(c.p, ux[5], c.q * uy[6]), p3b = mad_(c.q, ux[5], c.p * uy[6]);
  const T ts = uz[3] + uy[5] + ux[6];
  const T tts = c.t * ts;
  const T t1 = mad_(c.rmt, uz[3], tts), t2 = mad_(c.rmt, uy[5], tts), t3 = mad_(c.rmt, ux[6], tts);
  ux[0] = T(0); uy[0] = T(0); uz[0] = T(0);
  ux[1] = bxx; uy[1] = sxy; uz[1] = sxz;
  ux[2] = sxy; uy[2] = byy; uz[2] = syz;
  ux[3] = p1a; uy[3] = p2a; uz[3] = t1;
  ux[4] = sxz; uy[4] = syz; uz[4] = bzz;
  ux[5] = p3a; uy[5] = t2;  uz[5] = p2b;
  ux[6] = t3;  uy[6] = p3b; uz[6] = p1b;
  ux[7] *= c.w; uy[7] *= c.w; uz[7] *= c.w;
}

// Galerkin element of a level l >= 2, stored in the mode basis (modes in,
// modes out).  Restricting the level-1 moment matrices to a child keeps their
// joint pattern, so every deeper Galerkin element matrix lives on the same 279
// symmetric positions; it is held as its 150 entries with row <= col
// (kGMPairs), padded to TG_GM_STRIDE, in the 64-element blocks of gm_index.
// The entries are read in 16-byte pieces, a few pieces ahead of their use, so
// that few registers hold them at a time.  279 multiply-adds per element.
template <class T, int G = 4>   // G: pieces per group of loads in flight
__device__ __forceinline__ void elem_mode_stored(T* ux, T* uy, T* uz, const T* __restrict__ Km, int e) {
  constexpr int W = 16 / sizeof(T);                  // entries per piece
  constexpr int NP = TG_GM_STRIDE / W;               // pieces per element
  constexpr int NG = (NP + G - 1) / G;
  typedef T vecT __attribute__((ext_vector_type(W)));
  // piece p of element e at kp[64 p]
  const vecT* kp = (const vecT*)gp(Km) + (((long long)(e >> 6) * NP) << 6) + (e & 63);
  T a[24], y[24];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    a[3 * m + 0] = ux[m];
    a[3 * m + 1] = uy[m];
    a[3 * m + 2] = uz[m];
  }
#pragma unroll
  for (int r = 0; r < 24; ++r) y[r] = T(-0.0);
  vecT buf[2][G];
#pragma unroll
  for (int i = 0; i < G; ++i) buf[0][i] = kp[64 * i];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (g + 1 < NG) {
#pragma unroll
      for (int i = 0; i < G; ++i)
        if ((g + 1) * G + i < NP) buf[(g + 1) & 1][i] = kp[64 * ((g + 1) * G + i)];
    }
#pragma unroll
    for (int i = 0; i < G; ++i)
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int v = (g * G + i) * W + w;
        if (v < TG_GM_NU) {
          const int r = kGMPairs[v][0], c = kGMPairs[v][1];
          const T k = buf[g & 1][i][w];
          y[r] = mad_(k, a[c], y[r]);
          if (r != c) y[c] = mad_(k, a[r], y[c]);
        }
      }
    // Ordering point: the next group's loads are not issued before this
    // group's products are formed, which bounds the registers in use.
    asm volatile("" ::"v"(y[3]), "v"(y[4]), "v"(y[5]), "v"(y[6]), "v"(y[7]), "v"(y[8]), "v"(y[9]),
                 "v"(y[10]), "v"(y[11]), "v"(y[12]), "v"(y[13]), "v"(y[14]), "v"(y[15]), "v"(y[16]),
                 "v"(y[17]), "v"(y[18]), "v"(y[19]), "v"(y[20]), "v"(y[21]), "v"(y[22]), "v"(y[23]));
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    ux[m] = y[3 * m + 0];
    uy[m] = y[3 * m + 1];
    uz[m] = y[3 * m + 2];
  }
}

template <class T> __device__ __forceinline__ const T* G1V(const ProbDesc& P);
template <> __device__ __forceinline__ const double* G1V<double>(const ProbDesc& P) { return P.G1v64; }
template <> __device__ __forceinline__ const float* G1V<float>(const ProbDesc& P) { return P.G1v32; }

// Level-1 Galerkin element in moment form (modes in, modes out): with mu the
// eight Walsh moments of the children's moduli (mu_G = sum_c chi_G(c) E_c),
// sum_c E_c T_c^T Khat T_c = sum_G mu_G M_G, eight fixed matrices with 279
// nonzeros in all taking 21 distinct values (pattern kG1Pattern, values v from
// the host, held in scalar registers).  About 430 multiply-adds instead of
// eight child restrictions and contractions.
template <class T>
__device__ __forceinline__ void elem_galerkin1(T* ux, T* uy, T* uz, const T TG_GLOBAL* E0, int nx0, int ny0,
                                               int ex, int ey, int ez,
                                               const T __attribute__((address_space(4)))* v) {
  T mu[8];
  const long long base = 2LL * ex + (long long)nx0 * (2LL * ey + (long long)ny0 * 2LL * ez);
#pragma unroll
  for (int c = 0; c < 8; ++c)
    mu[c] = E0[base + (c & 1) + (long long)nx0 * (((c >> 1) & 1) + (long long)ny0 * (c >> 2))];
  wht_fwd(mu);
  T a[24], y[24];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    a[3 * m + 0] = ux[m];
    a[3 * m + 1] = uy[m];
    a[3 * m + 2] = uz[m];
  }
  // -0.0 is the exact additive identity, so untouched sums fold away
#pragma unroll
  for (int r = 0; r < 24; ++r) y[r] = T(-0.0);
#pragma unroll
  for (int G = 0; G < 8; ++G) {
    T t[24];
#pragma unroll
    for (int r = 0; r < 24; ++r) t[r] = T(-0.0);
#pragma unroll
    for (int e = 0; e < TG_G1_NNZ; ++e)
      if (kG1Pattern[e].g == G) t[kG1Pattern[e].r] = mad_(v[kG1Pattern[e].k], a[kG1Pattern[e].c], t[kG1Pattern[e].r]);
#pragma unroll
    for (int r = 0; r < 24; ++r)
      if ((kG1RowMask[G] >> r) & 1u) y[r] = mad_(mu[G], t[r], y[r]);
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    ux[m] = y[3 * m + 0];
    uy[m] = y[3 * m + 1];
    uz[m] = y[3 * m + 2];
  }
}

// ---------------------------------------------------------------------------
// BF16 matrix-core form of the fine element contraction v = Ke u (FP32
// accumulate, the element modulus applied to the FP32 result).  A wave's 64
// elements (4 rows of 16 element columns) are the columns N of four
// v_mfma_f32_16x16x32_bf16 products, one per element row; Ke (24 rows padded
// to 32, two 16-row tiles: bottom-face outputs, top-face outputs) is the A
// operand, held in registers for the whole kernel.  Lane layout of that
// instruction (measured on gfx950): A[i][k] at lane i % 16 + 16 (k / 8),
// element k % 8; B[k][n] at lane n + 16 (k / 8), element k % 8; D[m][n] at
// lane n + 16 (m / 4), element m % 4.  The K slots are laid out so that B
// comes straight from LDS: slot group g = k / 8 holds corners 2 g (s < 4) and
// 2 g + 1 (s >= 4), s = k % 8, component s % 4 (s % 4 = 3 is a zero pad), so
// lane n + 16 g reads two adjacent nodes of one node row: the (dj, dk) =
// (g & 1, g >> 1) row of element n's faces.  Node values are rounded to BF16
// once, when their layer is staged (hi = bf16(u); SPLIT adds
// lo = bf16(u - hi) and Ke_lo = bf16(Ke - Ke_hi):
// Ke_hi u_hi + Ke_hi u_lo + Ke_lo u_hi, about 16 significant bits).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

struct MfmaA {
  bf16x8 hi[2], lo[2];   // two 16-row tiles of Ke
};

__device__ __forceinline__ void mfma_load_ke(const float TG_GLOBAL* Ke, MfmaA& A) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      // tile mt holds Ke rows 12 mt .. 12 mt + 11 (bottom, then top face) and
      // four zero rows; K slot 8 g + s is DOF 3 (2 g + s / 4) + s % 4
      const int row = 12 * mt + i, comp = s & 3, col = 3 * (2 * g + (s >> 2)) + comp;
      const float v = (i < 12 && comp < 3) ? Ke[row * 24 + col] : 0.f;
      const __bf16 h = (__bf16)v;
      A.hi[mt][s] = h;
      A.lo[mt][s] = (__bf16)(v - (float)h);
    }
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// (x0, x1) rounded to BF16 and packed (x0 in the low half)
__device__ __forceinline__ unsigned pack_bf16(float x0, float x1) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){x0, x1}, bf16x2));
}

// One node's three components as B-operand words, (x, y) and (z, 0): the
// BF16 high parts into hi, and (SPLIT) the low parts into lo.
template <bool SPLIT>
__device__ __forceinline__ void split_node(float a0, float a1, float a2, uint2& hi, uint2& lo) {
  hi.x = pack_bf16(a0, a1);
  hi.y = pack_bf16(a2, 0.f);
  if (SPLIT) {
    // the exact remainders u - bf16(u), rounded to BF16
    const float h0 = __builtin_bit_cast(float, hi.x << 16);
    const float h1 = __builtin_bit_cast(float, hi.x & 0xffff0000u);
    const float h2 = __builtin_bit_cast(float, hi.y << 16);
    lo.x = pack_bf16(a0 - h0, a1 - h1);
    lo.y = pack_bf16(a2 - h2, 0.f);
  }
}

template <class T> __device__ __forceinline__ T* fpool(const LevelDesc& L);
template <> __device__ __forceinline__ double* fpool<double>(const LevelDesc& L) { return L.vec64; }
template <> __device__ __forceinline__ float* fpool<float>(const LevelDesc& L) { return L.vec32; }
template <class T> __device__ __forceinline__ const T* fE(const ProbDesc& P);
template <> __device__ __forceinline__ const double* fE<double>(const ProbDesc& P) { return P.E64; }
template <> __device__ __forceinline__ const float* fE<float>(const ProbDesc& P) { return P.E32; }
template <class T> __device__ __forceinline__ const T* fKm(const LevelDesc& L);
template <> __device__ __forceinline__ const double* fKm<double>(const LevelDesc& L) { return L.Km64; }
template <> __device__ __forceinline__ const float* fKm<float>(const LevelDesc& L) { return L.Km32; }
template <class T> __device__ __forceinline__ const T* fD(const LevelDesc& L);
template <> __device__ __forceinline__ const double* fD<double>(const LevelDesc& L) { return L.Dinv64; }
template <> __device__ __forceinline__ const float* fD<float>(const LevelDesc& L) { return L.Dinv32; }

template <class T>
__device__ __forceinline__ const T* fvec(const LevelDesc& L, int slot, const void* ext) {
  return slot < 0 ? (const T*)ext : fpool<T>(L) + (long long)slot * L.stride;
}

#define FZ_TX 16
#define FZ_OUT 15

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations
// (lgkmcnt) and synchronizes, leaving global loads in flight (a plain
// __syncthreads is a release fence that also drains every outstanding global
// load, which defeats prefetching one layer ahead).  The memory clobber keeps
// the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}


// z-tiles of height zc node layers
__host__ __device__ __forceinline__ int fz_tiles(int NX, int NY, int NZ, int zc) {
  return ((NX + FZ_OUT - 1) / FZ_OUT) * ((NY + FZ_OUT - 1) / FZ_OUT) * ((NZ + zc - 1) / zc);
}

// KIND 0: fine level, element = E_e Ke; KIND 1: level 1, matrix-free Galerkin
// (moment form); KIND 2 / 3: fine level with the BF16 matrix-core contraction
// (3: split BF16); KIND 4: level l >= 2, stored mode-basis Galerkin elements.
template <class T, int OP, int KIND, class TY = T>
__global__ __launch_bounds__(256) void k_fine_zm(const ProbDesc* __restrict__ probs,
                                                 const int2* __restrict__ work, int l, int sx,
                                                 const void* ex_, int sb, const void* eb_, int sy,
                                                 void* ey_, int sy2, T omega, ModeCoef<T> mc,
                                                 int vbskip) {
  // Single buffers suffice: every read of a layer's values happens between the
  // two barriers of its step, every write of the next layer after them.
  constexpr bool MF = (KIND == 2 || KIND == 3);   // matrix-core forms
  // node values of the current top layer; FP32 rows padded to 48 words so
  // that the two tile rows a half-wave touches fall in disjoint LDS banks
  // (17 columns of 16 consecutive reads per row)
  __shared__ T su[MF ? 1 : 3][17][sizeof(T) == 4 ? 48 : 17];
  // matrix-core forms: the BF16 high and low parts of two node layers (slot =
  // layer & 1: the bottom and the top face of the current element layer) and
  // the moduli of the current element layer
  __shared__ uint2 sbh[MF ? 2 : 1][17][17], sbl[KIND == 3 ? 2 : 1][17][17];
  __shared__ float sE[MF ? FZ_TX : 1][FZ_TX];
  // per element: 4 corners x 3 comps, layer sum (the matrix-core forms also
  // write four planes that are never read, from the padding rows of their
  // products)
  // (planes of 16 x 16; the matrix-core forms write lane groups g = 0..3 to
  // planes 4 g .. 4 g + 3, so their planes are padded to 260 words: the two
  // lane groups of a half-wave then use disjoint banks)
  constexpr int SSP = MF ? 260 : FZ_TX * FZ_TX;
  __shared__ T ss[MF ? 16 : 12][SSP];
  MfmaA mfA;
  const int2 wi = work[xcd_tile(blockIdx.x, gridDim.x)];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  // inside a V-cycle, levels from the problem's bottom level down belong to k_vbottom
  if ((KIND == 1 || KIND == 4) && vbskip && l >= (sizeof(T) == 8 ? P.vb_lb64 : P.vb_lb32)) return;
  const LevelDesc& L = P.lv[l];
  const int NX = L.NX, NY = L.NY, NZ = L.NZ, nx = L.ex, ny = L.ey, nz = L.ez;
  const int nx0 = P.lv[0].ex, ny0 = P.lv[0].ey;
  if constexpr (MF) mfma_load_ke(gp(P.Ke32), mfA);
  constexpr bool RST = (OP == FOP_RESTRICT);
  // coarse level (restriction only)
  const int NXc = RST ? P.lv[l + 1].NX : 0, NYc = RST ? P.lv[l + 1].NY : 0, NZc = RST ? P.lv[l + 1].NZ : 0;
  const int rzm = rz_layers(L.zc);
  const int ntx = RST ? (NXc + RZ_C - 1) / RZ_C : (NX + FZ_OUT - 1) / FZ_OUT;
  const int nty = RST ? (NYc + RZ_C - 1) / RZ_C : (NY + FZ_OUT - 1) / FZ_OUT;
  const int tile = wi.y;
  const int zc = L.zc;
  const int tiz = tile / (ntx * nty), rem = tile - tiz * ntx * nty;
  const int tiy = rem / ntx, tix = rem - tiy * ntx;
  const int x0 = RST ? 2 * RZ_C * tix - 1 : tix * FZ_OUT;
  const int y0 = RST ? 2 * RZ_C * tiy - 1 : tiy * FZ_OUT;
  const int z0 = RST ? 2 * rzm * tiz - 1 : tiz * zc;
  const int zend = RST ? min(2 * rzm * (tiz + 1), NZ) : min(z0 + zc, NZ);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int ex = x0 - 1 + tx, ey = y0 - 1 + ty;         // this thread's element column
  const int ni = ex + 1, nj = ey + 1;                   // this thread's node column
  const auto* u = gp(fvec<T>(L, sx, ex_));
  const auto* Eg = gp(fE<T>(P));
  const bool elem_in = (ex >= 0 && ex < nx && ey >= 0 && ey < ny);
  const bool owner = (tx < FZ_OUT && ty < FZ_OUT && ni < NX && nj < NY);
  // fine residuals of the restriction tile, coarse accumulators of its 7 x 7
  // coarse columns (threads 0..48)
  __shared__ T rl[RST ? 3 : 1][FZ_OUT][FZ_OUT];
  T racc[3] = {T(0), T(0), T(0)};
  // extra node loads: tile row/column 0 (nodes x0-1 or y0-1)
  const int xt = threadIdx.x;
  int exi = -1, exj = -1, etx = 0, ety = 0;
  if (xt < 17) { etx = 0; ety = xt; exi = x0 - 1; exj = y0 - 1 + xt; }
  else if (xt < 33) { etx = xt - 16; ety = 0; exi = x0 - 1 + (xt - 16); exj = y0 - 1; }
  const bool own_col = (ni > 0 && ni < NX && nj >= 0 && nj < NY);
  const bool ext_col = (xt < 33) && (exi > 0 && exi < NX && exj >= 0 && exj < NY);
  const long long own_base = 3LL * (ni + (long long)NX * nj);
  const long long ext_base = 3LL * (exi + (long long)NX * exj);
  const long long lstride = 3LL * NX * NY;             // DOFs per node layer

  // prefetch registers for one node layer (own column + extra column),
  // returned by value so they stay in registers
  struct Pre {
    T a0, a1, a2, e0, e1, e2;
    T b0, b1, b2;              // FOP_SMOOTH1: b at the own node
  };
  constexpr bool S1 = (OP == FOP_SMOOTH1);
  const double in_scale = (S1 && sx >= 0) ? P.small[sx] : 1.0;
  // FOP_SMOOTH1: b at node (column base, layer k) from the FP64 slot, scaled,
  // and the first sweep x = w D^-1 b there
  auto first_sweep = [&](long long base, int k, T& x0, T& x1, T& x2, T& c0, T& c1, T& c2) {
    const double TG_GLOBAL* bp = gp(P.lv[0].vec64 + (long long)sb * L.stride) + base + lstride * k;
    c0 = T(bp[0] * in_scale);
    c1 = T(bp[1] * in_scale);
    c2 = T(bp[2] * in_scale);
    const T TG_GLOBAL* Dp = gp(fD<T>(L)) + 9 * (base / 3 + (lstride / 3) * k);
    x0 = omega * mad_(Dp[2], c2, mad_(Dp[1], c1, Dp[0] * c0));
    x1 = omega * mad_(Dp[5], c2, mad_(Dp[4], c1, Dp[3] * c0));
    x2 = omega * mad_(Dp[8], c2, mad_(Dp[7], c1, Dp[6] * c0));
  };
  auto fetch = [&](int k) -> Pre {
    Pre r;
    r.b0 = r.b1 = r.b2 = T(0);
    const bool kin = (k >= 0 && k < NZ);
    if (S1) {
      T c0, c1, c2;
      if (own_col && kin) {
        first_sweep(own_base, k, r.a0, r.a1, r.a2, r.b0, r.b1, r.b2);
      } else {
        r.a0 = r.a1 = r.a2 = T(0);
      }
      if (ext_col && kin) {
        first_sweep(ext_base, k, r.e0, r.e1, r.e2, c0, c1, c2);
      } else {
        r.e0 = r.e1 = r.e2 = T(0);
      }
      return r;
    }
    if (own_col && kin) {
      const auto* p = u + own_base + lstride * k;
      r.a0 = p[0];
      r.a1 = p[1];
      r.a2 = p[2];
    } else {
      r.a0 = r.a1 = r.a2 = T(0);
    }
    if (ext_col && kin) {
      const auto* p = u + ext_base + lstride * k;
      r.e0 = p[0];
      r.e1 = p[1];
      r.e2 = p[2];
    } else {
      r.e0 = r.e1 = r.e2 = T(0);
    }
    return r;
  };
  auto stage = [&](const Pre& r, int k) {
    if constexpr (MF) {
      constexpr bool SPL = KIND == 3;
      split_node<SPL>(r.a0, r.a1, r.a2, sbh[k & 1][ty + 1][tx + 1], sbl[SPL ? k & 1 : 0][ty + 1][tx + 1]);
      if (xt < 33) split_node<SPL>(r.e0, r.e1, r.e2, sbh[k & 1][ety][etx], sbl[SPL ? k & 1 : 0][ety][etx]);
    } else {
      su[0][ty + 1][tx + 1] = r.a0;
      su[1][ty + 1][tx + 1] = r.a1;
      su[2][ty + 1][tx + 1] = r.a2;
      if (xt < 33) {
        su[0][ety][etx] = r.e0;
        su[1][ety][etx] = r.e1;
        su[2][ety][etx] = r.e2;
      }
    }
  };
  // State carried from one element layer to the next: the shared face in the
  // form the contraction takes it (face-mode for the vector forms, raw node
  // values for the matrix-core forms), the previous layer's top-face outputs,
  // the raw value of node (ni, nj, k) for the smoother and the next layer's
  // modulus.  The vector forms unroll the march by two with the roles of two
  // such states alternating, so nothing is copied between layers.
  struct St {
    T bx[4], by[4], bz[4];     // bottom face, corner c = di + 2 dj
    T tpx[4], tpy[4], tpz[4];  // top-face outputs of the previous element layer
    T own[3];
    T bo[3];                   // FOP_SMOOTH1: b at node (ni, nj, k)
    T E;
    T cr[16];                  // matrix-core forms: the same outputs in the D layout
  };
  St s0, s1;
#pragma unroll
  for (int c = 0; c < 4; ++c) s0.tpx[c] = s0.tpy[c] = s0.tpz[c] = T(0);
#pragma unroll
  for (int q = 0; q < 16; ++q) s0.cr[q] = T(0);
  Pre pre = fetch(z0 - 1);
  stage(pre, z0 - 1);
  s0.bo[0] = pre.b0;
  s0.bo[1] = pre.b1;
  s0.bo[2] = pre.b2;
  if constexpr (MF) {
    // node (ni, nj, z0 - 1) of this thread; the face stays in LDS
    s0.own[0] = pre.a0;
    s0.own[1] = pre.a1;
    s0.own[2] = pre.a2;
  }
  pre = fetch(z0);           // in flight while the prologue reads LDS
  lds_barrier();
  if constexpr (!MF) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int di = c & 1, dj = c >> 1;
      s0.bx[c] = su[0][ty + dj][tx + di];
      s0.by[c] = su[1][ty + dj][tx + di];
      s0.bz[c] = su[2][ty + dj][tx + di];
    }
    s0.own[0] = s0.bx[3];
    s0.own[1] = s0.by[3];
    s0.own[2] = s0.bz[3];
    face_fwd(s0.bx);
    face_fwd(s0.by);
    face_fwd(s0.bz);
  }
  const ModeCoefE<T> mce = {mc.d - mc.o, mc.o, mc.s, mc.p, mc.q, mc.r - mc.t, mc.t, mc.w};
  // element moduli of this column: index ecol + elay * k for element layer k
  const long long ecol = ex + (long long)nx * ey, elay = (long long)nx * ny;
  auto modulus = [&](int k) -> T {
    return ((KIND == 0 || MF) && elem_in && k >= 0 && k < nz) ? Eg[ecol + elay * k] : T(0);
  };
  s0.E = modulus(z0 - 1);
  lds_barrier();           // prologue reads done before the first layer is staged

  // one element layer k: A holds the state entering it, B receives the state
  // for layer k + 1
  auto step = [&](const int k, St& A, St& B) {
    const T own0 = A.own[0], own1 = A.own[1], own2 = A.own[2];   // node (ni, nj, k)
    if constexpr (MF) {
      B.own[0] = pre.a0;     // node (ni, nj, k + 1)
      B.own[1] = pre.a1;
      B.own[2] = pre.a2;
    }
    // (A and B may be one object: read A's b before B's is written)
    const T bo0 = A.bo[0], bo1 = A.bo[1], bo2 = A.bo[2];   // b at node (ni, nj, k)
    if constexpr (S1) {
      B.bo[0] = pre.b0;      // b at node (ni, nj, k + 1)
      B.bo[1] = pre.b1;
      B.bo[2] = pre.b2;
    }
    stage(pre, k + 1);       // node layer k + 1 (fetched one step ahead)
    pre = fetch(k + 2);      // next layer in flight during this step
    const T Ecur = A.E;      // modulus of element layer k (0 outside the grid)
    if constexpr (MF) sE[ty][tx] = (float)Ecur;
    B.E = modulus(k + 1);
    // output-side operands of node (ni, nj, k), loaded before the barrier
    T rb0 = T(0), rb1 = T(0), rb2 = T(0);
    T D[9];
    const bool out_now = owner && own_col && k >= z0 && k >= 0;
    const long long n = ni + (long long)NX * (nj + (long long)NY * k);
    if (S1) {
      rb0 = bo0; rb1 = bo1; rb2 = bo2;
    } else if (OP != FOP_APPLY && out_now) {
      const auto* bb = gp(fvec<T>(L, sb, eb_)) + 3 * n;
      rb0 = bb[0]; rb1 = bb[1]; rb2 = bb[2];
    }
    if ((OP == FOP_SMOOTH || S1) && out_now) {
      const auto* Dp = gp(fD<T>(L)) + 9 * n;
#pragma unroll
      for (int q = 0; q < 9; ++q) D[q] = Dp[q];
    }
    lds_barrier();
    T ux[8], uy[8], uz[8];
    const bool ein = elem_in && k >= 0 && k < nz;
    if constexpr (!MF) {
      T fx[4], fy[4], fz[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int di = c & 1, dj = c >> 1;
        fx[c] = su[0][ty + dj][tx + di];
        fy[c] = su[1][ty + dj][tx + di];
        fz[c] = su[2][ty + dj][tx + di];
      }
      B.own[0] = fx[3];
      B.own[1] = fy[3];
      B.own[2] = fz[3];
      face_fwd(fx);
      face_fwd(fy);
      face_fwd(fz);
      // z stage of the mode transform; the top face becomes the next bottom face
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        ux[c] = A.bx[c] + fx[c];
        ux[c + 4] = fx[c] - A.bx[c];
        uy[c] = A.by[c] + fy[c];
        uy[c + 4] = fy[c] - A.by[c];
        uz[c] = A.bz[c] + fz[c];
        uz[c + 4] = fz[c] - A.bz[c];
        B.bx[c] = fx[c];
        B.by[c] = fy[c];
        B.bz[c] = fz[c];
      }
      if constexpr (KIND == 0) {
        mode_contract_e(ux, uy, uz, coef_times(mce, Ecur));
      } else if (KIND == 1 && ein) {
        // read-only table: constant address space, so the loads are scalar
        elem_galerkin1<T>(ux, uy, uz, Eg, nx0, ny0, ex, ey, k,
                          (const T __attribute__((address_space(4)))*)G1V<T>(P));
      } else if (KIND == 4 && ein) {
        elem_mode_stored<T>(ux, uy, uz, fKm<T>(L), (int)(ecol + elay * k));
      } else {
#pragma unroll
        for (int a = 0; a < 8; ++a) ux[a] = uy[a] = uz[a] = T(0);
      }
      // inverse z stage; face k = bottom of this element + top of the previous
      // one, summed in face-mode form, then the face's inverse x, y stages
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        fx[c] = (ux[c] - ux[c + 4]) + A.tpx[c];
        fy[c] = (uy[c] - uy[c + 4]) + A.tpy[c];
        fz[c] = (uz[c] - uz[c + 4]) + A.tpz[c];
        B.tpx[c] = ux[c] + ux[c + 4];
        B.tpy[c] = uy[c] + uy[c + 4];
        B.tpz[c] = uz[c] + uz[c + 4];
      }
      face_inv(fx);
      face_inv(fy);
      face_inv(fz);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        ss[3 * c + 0][ty * FZ_TX + tx] = fx[c];
        ss[3 * c + 1][ty * FZ_TX + tx] = fy[c];
        ss[3 * c + 2][ty * FZ_TX + tx] = fz[c];
      }
    } else {
      // lane n + 16 g of wave w works on element (n, 4 w + nb) of the tile for
      // nb = 0..3: its B operand is node row (dj, dk) = (g & 1, g >> 1) of that
      // element's faces, two adjacent nodes, read as staged
      const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15, r0 = 4 * (threadIdx.x >> 6);
      const int dj = g & 1, sl = (k + (g >> 1)) & 1;
      float Ev[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) Ev[nb] = sE[r0 + nb][n];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const uint2 h0 = sbh[sl][r0 + nb + dj][n], h1 = sbh[sl][r0 + nb + dj][n + 1];
        const bf16x8 bh = __builtin_bit_cast(bf16x8, (u32x4){h0.x, h0.y, h1.x, h1.y});
        f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
        c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mfA.hi[0], bh, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mfA.hi[1], bh, c1, 0, 0, 0);
        if constexpr (KIND == 3) {
          const uint2 l0 = sbl[sl][r0 + nb + dj][n], l1 = sbl[sl][r0 + nb + dj][n + 1];
          const bf16x8 bl = __builtin_bit_cast(bf16x8, (u32x4){l0.x, l0.y, l1.x, l1.y});
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mfA.hi[0], bl, c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mfA.hi[1], bl, c1, 0, 0, 0);
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mfA.lo[0], bh, c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mfA.lo[1], bh, c1, 0, 0, 0);
        }
        // lane n + 16 g, component w: face DOF 4 g + w (g < 3) of element
        // (n, r0 + nb); layer-k nodes get this element's bottom face plus the
        // previous element layer's top face, scaled by the moduli
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          ss[4 * g + w][(r0 + nb) * FZ_TX + n] = mad_(Ev[nb], c0[w], (float)A.cr[4 * nb + w]);
          B.cr[4 * nb + w] = T(Ev[nb] * c1[w]);
        }
      }
    }
    lds_barrier();
    // (the restriction needs every fine column of its tile, zero outside the grid)
    if ((RST ? (tx < FZ_OUT && ty < FZ_OUT) : owner) && k >= z0) {
      // node (ni, nj, k) = corner 3 of element (tx,ty), corner 2 of (tx+1,ty),
      // corner 1 of (tx,ty+1), corner 0 of (tx+1,ty+1)
      T a[3];
#pragma unroll
      for (int q = 0; q < 3; ++q)
        a[q] = (ss[9 + q][ty * FZ_TX + tx] + ss[6 + q][ty * FZ_TX + tx + 1]) +
               (ss[3 + q][(ty + 1) * FZ_TX + tx] + ss[0 + q][(ty + 1) * FZ_TX + tx + 1]);
      if constexpr (RST) {
        // free-DOF residual; zero at clamped nodes and outside the grid
#pragma unroll
        for (int q = 0; q < 3; ++q) rl[q][ty][tx] = out_now ? (q == 0 ? rb0 : q == 1 ? rb1 : rb2) - a[q] : T(0);
      } else {
      auto* y = gp((sy < 0 ? (TY*)ey_ : fpool<TY>(L) + (long long)sy * L.stride)) + 3 * n;
      if constexpr (S1) {
        // the FP32 copy of b for the later sweeps (zero at clamped nodes)
        auto* bt = gp(fpool<T>(L) + (long long)sy2 * L.stride) + 3 * n;
        bt[0] = rb0;
        bt[1] = rb1;
        bt[2] = rb2;
      }
      if (ni == 0) {
        y[0] = y[1] = y[2] = TY(0);
      } else if (OP == FOP_APPLY) {
        y[0] = TY(a[0]);
        y[1] = TY(a[1]);
        y[2] = TY(a[2]);
      } else {
        const T r0 = rb0 - a[0], r1 = rb1 - a[1], r2 = rb2 - a[2];
        if (OP == FOP_RESID) {
          y[0] = TY(r0);
          y[1] = TY(r1);
          y[2] = TY(r2);
        } else {
          y[0] = TY(mad_(omega, mad_(D[2], r2, mad_(D[1], r1, D[0] * r0)), own0));
          y[1] = TY(mad_(omega, mad_(D[5], r2, mad_(D[4], r1, D[3] * r0)), own1));
          y[2] = TY(mad_(omega, mad_(D[8], r2, mad_(D[7], r1, D[6] * r0)), own2));
        }
      }
      }
    }
    if constexpr (RST) {
      lds_barrier();
      if (k >= z0 && threadIdx.x < RZ_C * RZ_C) {
        // 3 x 3 in-layer part of the full weighting around fine node
        // (1 + 2 il, 1 + 2 jl) of the tile, then the layer's weight for the
        // coarse layers it touches: 1 for K = k / 2 (k even), 1/2 for
        // K = (k -+ 1) / 2 (k odd); coarse layer (k - 1) / 2 is complete after
        // odd layer k, the last coarse layer after the last fine layer
        const int il = threadIdx.x % RZ_C, jl = threadIdx.x / RZ_C;
        T sxy[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
          for (int di = -1; di <= 1; ++di) {
            const T w = T(1) / T(1 << ((dj != 0) + (di != 0)));
#pragma unroll
            for (int q = 0; q < 3; ++q) sxy[q] = mad_(w, rl[q][1 + 2 * jl + dj][1 + 2 * il + di], sxy[q]);
          }
        int K = -1;
        if (k & 1) {
#pragma unroll
          for (int q = 0; q < 3; ++q) racc[q] = mad_(T(0.5), sxy[q], racc[q]);
          K = (k - 1) / 2;
        } else {
#pragma unroll
          for (int q = 0; q < 3; ++q) racc[q] += sxy[q];
          if (k == NZ - 1) K = k / 2;
        }
        const int I = RZ_C * tix + il, J = RZ_C * tiy + jl;
        if (K >= rzm * tiz && K < NZc && I < NXc && J < NYc) {
          const LevelDesc& Lc = P.lv[l + 1];
          auto* bc = gp(fpool<TY>(Lc) + (long long)sy * Lc.stride) + 3 * (I + (long long)NXc * (J + (long long)NYc * K));
          T bv[3];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            bv[q] = I == 0 ? T(0) : racc[q];   // coarse x = 0 clamped
            bc[q] = TY(bv[q]);
          }
          if (sy2 >= 0 && l + 1 < P.nlev - 1) {
            // the coarse level's first Jacobi sweep from zero, x = w D^-1 b
            const long long nc = I + (long long)NXc * (J + (long long)NYc * K);
            const auto* Dc = gp(fD<T>(Lc)) + 9 * nc;
            auto* xc = gp(fpool<TY>(Lc) + (long long)sy2 * Lc.stride) + 3 * nc;
#pragma unroll
            for (int q = 0; q < 3; ++q)
              xc[q] = TY(omega * mad_(Dc[3 * q + 2], bv[2], mad_(Dc[3 * q + 1], bv[1], Dc[3 * q] * bv[0])));
          }
        }
        if (k & 1) {
#pragma unroll
          for (int q = 0; q < 3; ++q) racc[q] = T(0.5) * sxy[q];
        }
      }
    }
  };
  if constexpr (MF || KIND == 4 || sizeof(T) == 8) {
    // register-bound forms (and FP64): one state, updated in place
    for (int k = z0 - 1; k < zend; ++k) step(k, s0, s0);
  } else {
    int k = z0 - 1;
    for (; k + 1 < zend; k += 2) {
      step(k, s0, s1);
      step(k + 1, s1, s0);
    }
    if (k < zend) step(k, s0, s1);
  }
}

// ---------------------------------------------------------------------------
// host side: mode coefficients from Ke, launches
// K_H = T Ke T^T with T = kron(H8, I3), H8[m][a] = prod over set bits b of m of
// (2 a_b - 1).  For a cube the only nonzeros are the 8-coefficient pattern
// used by elem_mode_apply; anything else is an error.
int mode_coef_from_ke(const double* Ke, ModeCoef<double>* out64, ModeCoef<float>* out32) {
  double H[8][8];
  for (int m = 0; m < 8; ++m)
    for (int a = 0; a < 8; ++a) {
      double v = 1.0;
      for (int b = 0; b < 3; ++b)
        if (m & (1 << b)) v *= ((a >> b) & 1) ? 1.0 : -1.0;
      H[m][a] = v;
    }
  double KH[24][24];
  for (int r = 0; r < 24; ++r)
    for (int c = 0; c < 24; ++c) {
      double s = 0.0;
      const int mr = r / 3, cr = r % 3, mc = c / 3, cc = c % 3;
      for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) s += H[mr][a] * Ke[(3 * a + cr) * 24 + 3 * b + cc] * H[mc][b];
      KH[r][c] = s;
    }
  auto R = [](int m, int c) { return 3 * m + c; };
  ModeCoef<double> k;
  k.d = KH[R(1, 0)][R(1, 0)];
  k.o = KH[R(1, 0)][R(2, 1)];
  k.s = KH[R(1, 1)][R(1, 1)];
  k.p = KH[R(3, 0)][R(3, 0)];
  k.q = KH[R(3, 0)][R(6, 2)];
  k.r = KH[R(3, 2)][R(3, 2)];
  k.t = KH[R(3, 2)][R(5, 1)];
  k.w = KH[R(7, 0)][R(7, 0)];
  // rebuild the pattern and compare
  double P[24][24] = {};
  const int nrm[3] = {R(1, 0), R(2, 1), R(4, 2)};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[nrm[i]][nrm[j]] = (i == j) ? k.d : k.o;
  const int sh[3][2] = {{R(1, 1), R(2, 0)}, {R(1, 2), R(4, 0)}, {R(2, 2), R(4, 1)}};
  for (auto& pr : sh)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) P[pr[i]][pr[j]] = k.s;
  const int b1[3][2] = {{R(3, 0), R(6, 2)}, {R(3, 1), R(5, 2)}, {R(5, 0), R(6, 1)}};
  for (auto& pr : b1)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) P[pr[i]][pr[j]] = (i == j) ? k.p : k.q;
  const int b2[3] = {R(3, 2), R(5, 1), R(6, 0)};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[b2[i]][b2[j]] = (i == j) ? k.r : k.t;
  for (int c = 0; c < 3; ++c) P[R(7, c)][R(7, c)] = k.w;
  double mx = 0.0, err = 0.0;
  for (int r = 0; r < 24; ++r)
    for (int c = 0; c < 24; ++c) {
      mx = std::fmax(mx, std::fabs(KH[r][c]));
      err = std::fmax(err, std::fabs(KH[r][c] - P[r][c]));
    }
  if (err > 1e-12 * mx) return fail(TG_EINVAL, "element stiffness does not have the cube mode-basis pattern");
  const double sc = 1.0 / 64.0;
  const ModeCoef<double> m64 = {k.d * sc, k.o * sc, k.s * sc, k.p * sc, k.q * sc, k.r * sc, k.t * sc, k.w * sc};
  *out64 = m64;
  *out32 = {(float)m64.d, (float)m64.o, (float)m64.s, (float)m64.p,
            (float)m64.q, (float)m64.r, (float)m64.t, (float)m64.w};
  return TG_OK;
}

// Level-1 moment matrices M_G = (1/8) sum_c chi_G(c) T_c^T Khat T_c (the
// children c of a coarse element, T_c the per-dimension restriction
// (a0, a1) -> (a0 + s a1, a1 / 2), s = -1/2 or +1/2, Khat = T Ke T^T / 64), read
// out at the pattern kG1Pattern (one value per class of equal entries);
// entries outside it must vanish.
int galerkin1_values(const double* Ke, double* out) {
  double H[8][8];
  for (int m = 0; m < 8; ++m)
    for (int a = 0; a < 8; ++a) {
      double v = 1.0;
      for (int b = 0; b < 3; ++b)
        if (m & (1 << b)) v *= ((a >> b) & 1) ? 1.0 : -1.0;
      H[m][a] = v;
    }
  std::vector<double> Kh(576, 0.0);   // Khat, index 3 m + comp
  for (int r = 0; r < 24; ++r)
    for (int c = 0; c < 24; ++c) {
      double s = 0.0;
      const int mr = r / 3, cr = r % 3, mc = c / 3, cc = c % 3;
      for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) s += H[mr][a] * Ke[(3 * a + cr) * 24 + 3 * b + cc] * H[mc][b];
      Kh[r * 24 + c] = s / 64.0;
    }
  std::vector<double> M(8 * 576, 0.0), T(576), KT(576);
  for (int c = 0; c < 8; ++c) {
    // T_c: 24 x 24 on index 3 m + comp; per dimension b the 2x2 block
    // [[1, s_b], [0, 1/2]] on (bit b clear, bit b set)
    double sd[3];
    for (int b = 0; b < 3; ++b) sd[b] = ((c >> b) & 1) ? 0.5 : -0.5;
    for (int r = 0; r < 24; ++r)
      for (int q = 0; q < 24; ++q) {
        // child mode r / 3 from coarse mode q / 3, same component: per
        // dimension t(0,0) = 1, t(0,1) = s, t(1,1) = 1/2, t(1,0) = 0
        const int mr = r / 3, mq = q / 3;
        double v = (r % 3 == q % 3) ? 1.0 : 0.0;
        for (int b = 0; b < 3; ++b) {
          const int br = (mr >> b) & 1, bq = (mq >> b) & 1;
          v *= br ? (bq ? 0.5 : 0.0) : (bq ? sd[b] : 1.0);
        }
        T[r * 24 + q] = v;
      }
    for (int r = 0; r < 24; ++r)
      for (int q = 0; q < 24; ++q) {
        double s = 0.0;
        for (int t = 0; t < 24; ++t) s += Kh[r * 24 + t] * T[t * 24 + q];
        KT[r * 24 + q] = s;
      }
    for (int G = 0; G < 8; ++G) {
      double chi = 1.0;
      for (int b = 0; b < 3; ++b)
        if ((G >> b) & 1) chi *= ((c >> b) & 1) ? 1.0 : -1.0;
      for (int r = 0; r < 24; ++r)
        for (int q = 0; q < 24; ++q) {
          double s = 0.0;
          for (int t = 0; t < 24; ++t) s += T[t * 24 + r] * KT[t * 24 + q];
          M[G * 576 + r * 24 + q] += chi * s / 8.0;
        }
    }
  }
  std::vector<char> in(8 * 576, 0), set(TG_G1_NVAL, 0);
  for (int e = 0; e < TG_G1_NNZ; ++e) {
    const G1Entry& p = kG1Pattern[e];
    if (!set[p.k]) out[p.k] = M[p.g * 576 + p.r * 24 + p.c];
    set[p.k] = 1;
    in[p.g * 576 + p.r * 24 + p.c] = 1;
  }
  double mx = 0.0, err = 0.0;
  for (int q = 0; q < 8 * 576; ++q) mx = std::fmax(mx, std::fabs(M[q]));
  for (int q = 0; q < 8 * 576; ++q)
    if (!in[q]) err = std::fmax(err, std::fabs(M[q]));
  for (int e = 0; e < TG_G1_NNZ; ++e) {
    const G1Entry& p = kG1Pattern[e];
    err = std::fmax(err, std::fabs(M[p.g * 576 + p.r * 24 + p.c] - out[p.k]));
  }
  if (err > 1e-12 * mx) return fail(TG_EINVAL, "level-1 Galerkin moments fall outside the cube pattern");
  return TG_OK;
}

// Balanced height for a column of NZ node layers with at most zmax per tile.
int zm_height(int NZ, int zmax) {
  const int ntz = (NZ + zmax - 1) / zmax;
  return (NZ + ntz - 1) / ntz;
}
int zm_tiles(const tg_grid* g, int l, int zmax) {
  const int NZ = g->lv[l].ez + 1;
  return fz_tiles(g->lv[l].ex + 1, g->lv[l].ey + 1, NZ, zm_height(NZ, zmax));
}
// tiles of the fused residual-restriction sweep on level l (l + 1 must exist)
int rz_tiles(const tg_grid* g, int l, int zmax) {
  const int m = rz_layers(zm_height(g->lv[l].ez + 1, zmax));
  const int NXc = g->lv[l + 1].ex + 1, NYc = g->lv[l + 1].ey + 1, NZc = g->lv[l + 1].ez + 1;
  return ((NXc + RZ_C - 1) / RZ_C) * ((NYc + RZ_C - 1) / RZ_C) * ((NZc + m - 1) / m);
}

// Per level, the tallest z-tile in {16, 12, 8, 6, 4} that gives >= 2048
// workgroups over the whole batch, else 4.  Every tile recomputes one element
// layer, so taller tiles do less redundant work; shorter tiles give more
// parallelism.
void batch_choose_zc(Batch* b) {
  const int cand[5] = {16, 12, 8, 6, 4};
  for (int l = 0; l < TG_MAXLEV; ++l) {
    int pick = 4;
    for (int c : cand) {
      long long tiles = 0;
      for (auto* g : b->grids)
        if (l < g->nlev) tiles += zm_tiles(g, l, c);
      if (tiles >= 2048) {
        pick = c;
        break;
      }
    }
    b->zc[l] = pick;
  }
}

template <class T> static ModeCoef<T> mcoef(const tg_grid* g);
template <> ModeCoef<double> mcoef<double>(const tg_grid* g) { return g->mc64; }
template <> ModeCoef<float> mcoef<float>(const tg_grid* g) { return g->mc32; }

// OP: 0 apply, 1 residual, 2 smoothing sweep on level l with the z-march
// kernel (level 0: E Ke; levels 1..TG_MF_LEVELS: matrix-free Galerkin; deeper
// levels: stored mode-basis Galerkin elements).
// Every grid of a batch shares one Ke (checked at batch creation).
template <class T>
int launch_fine(const Batch* b, const DevList& dl, int l, int op, int sx, const void* ex, int sb,
                const void* eb, int sy, void* ey, double omega, hipStream_t s, int sy2, int vbskip) {
  if (!dl.n) return TG_OK;
  const ModeCoef<T> mc = mcoef<T>(b->grids[0]);
  const ProbDesc* desc = b->desc_d;
  const T om = T(omega);
#define TG_ZM(KV)                                                                                         \
  do {                                                                                                    \
    if (op == FOP_APPLY)                                                                                  \
      k_fine_zm<T, FOP_APPLY, KV><<<dl.n, 256, 0, s>>>(desc, dl.ptr, l, sx, ex, sb, eb, sy, ey, sy2, om, mc, vbskip);    \
    else if (op == FOP_RESID)                                                                             \
      k_fine_zm<T, FOP_RESID, KV><<<dl.n, 256, 0, s>>>(desc, dl.ptr, l, sx, ex, sb, eb, sy, ey, sy2, om, mc, vbskip);    \
    else if (op == FOP_SMOOTH)                                                                            \
      k_fine_zm<T, FOP_SMOOTH, KV><<<dl.n, 256, 0, s>>>(desc, dl.ptr, l, sx, ex, sb, eb, sy, ey, sy2, om, mc, vbskip);   \
    else if (op == FOP_SMOOTH1)                                                                           \
      k_fine_zm<T, FOP_SMOOTH1, KV><<<dl.n, 256, 0, s>>>(desc, dl.ptr, l, sx, ex, sb, eb, sy, ey, sy2, om, mc, vbskip);  \
    else                                                                                                  \
      k_fine_zm<T, FOP_RESTRICT, KV><<<dl.n, 256, 0, s>>>(desc, dl.ptr, l, sx, ex, sb, eb, sy, ey, sy2, om, mc, vbskip); \
  } while (0)
  if (op == FOP_SMOOTH1 && l != 0) return fail(TG_EINVAL, "the fused first sweeps are a level-0 operation");
  if (l == 0)
    TG_ZM(0);
  else if (l <= TG_MF_LEVELS)
    TG_ZM(1);
  else
    TG_ZM(4);
#undef TG_ZM
  return TG_OK;
}
template int launch_fine<double>(const Batch*, const DevList&, int, int, int, const void*, int, const void*,
                                 int, void*, double, hipStream_t, int, int);

// Level 0 with the BF16 matrix-core contraction (FP32 vectors): op as above.
int launch_fine_mfma(const Batch* b, const DevList& dl, int op, bool split, int sx, const void* ex, int sb,
                     const void* eb, int sy, void* ey, double omega, bool out64, hipStream_t s, int sy2) {
  if (!dl.n) return TG_OK;
  const ModeCoef<float> mc = mcoef<float>(b->grids[0]);
  const ProbDesc* desc = b->desc_d;
  const float om = float(omega);
#define TG_MF(OPV, K, TYV) \
  k_fine_zm<float, OPV, K, TYV><<<dl.n, 256, 0, s>>>(desc, dl.ptr, 0, sx, ex, sb, eb, sy, ey, sy2, om, mc, 0)
  if (out64) {
    if (split) TG_MF(FOP_SMOOTH, 3, double); else TG_MF(FOP_SMOOTH, 2, double);
  } else if (op == FOP_APPLY) {
    if (split) TG_MF(FOP_APPLY, 3, float); else TG_MF(FOP_APPLY, 2, float);
  } else if (op == FOP_RESID) {
    if (split) TG_MF(FOP_RESID, 3, float); else TG_MF(FOP_RESID, 2, float);
  } else if (op == FOP_SMOOTH) {
    if (split) TG_MF(FOP_SMOOTH, 3, float); else TG_MF(FOP_SMOOTH, 2, float);
  } else if (op == FOP_SMOOTH1) {
    if (split) TG_MF(FOP_SMOOTH1, 3, float); else TG_MF(FOP_SMOOTH1, 2, float);
  } else {
    if (split) TG_MF(FOP_RESTRICT, 3, float); else TG_MF(FOP_RESTRICT, 2, float);
  }
#undef TG_MF
  return TG_OK;
}

// Level-0 smoothing sweep whose output goes to an FP64 slot (the V-cycle's
// last post-sweep writing the Krylov vector z_j directly).
int launch_fine_smooth_out64(const Batch* b, const DevList& dl, int sx, int sb, int sy, double omega,
                             hipStream_t s) {
  if (!dl.n) return TG_OK;
  const ModeCoef<float> mc = mcoef<float>(b->grids[0]);
  k_fine_zm<float, FOP_SMOOTH, 0, double><<<dl.n, 256, 0, s>>>(b->desc_d, dl.ptr, 0, sx, nullptr, sb, nullptr,
                                                               sy, nullptr, -1, float(omega), mc, 0);
  return TG_OK;
}
template int launch_fine<float>(const Batch*, const DevList&, int, int, int, const void*, int, const void*,
                                int, void*, double, hipStream_t, int, int);

// ---------------------------------------------------------------------------
// The bottom of the V-cycle in one launch.  From a level lb >= 2 down, every
// level of a problem is small: one workgroup per problem keeps the level
// vectors x and b of levels lb..L in LDS and runs that part of the cycle
// (the remaining pre-sweeps, residual and restriction, the coarsest solve
// with the explicit inverse, prolongation and post-sweeps) with barriers in
// place of launches.  The level operators are the stored mode-basis Galerkin
// elements: an element pass writes each element's 24 outputs to LDS
// (component-major, one thread per element), a node pass sums the up to
// eight contributions of each node in a fixed order.  Entry: b and
// the first sweep x = w D^-1 b of level lb in slots C_B and C_XA (written by
// the restriction from level lb - 1; b only when lb is the coarsest level);
// exit: the level-lb result in slot sfin.
// threads per workgroup: FP32 fits 128 registers (16 waves), FP64 takes 256
// threads per workgroup (FP32 fits 128 registers with 16 waves, FP64 takes
// 256 with 8) and pieces of a stored element matrix in flight per group of
// loads (measured: all 38 FP32 pieces at once with 512 threads is no faster)
template <class T, bool L1>
struct VbThreads {
  static constexpr int N = sizeof(T) == 8 ? 512 : 1024;
  static constexpr int G = 8;
};

// LDS words (of type T) the bottom needs from level lb of grid g down
static size_t vb_words(const tg_grid* g, int lb) {
  const auto& H = g->lv[lb];
  size_t w = (size_t)24 * H.n_elem;                     // element outputs
  w += 3 * (size_t)H.n_nodes;                           // residual
  for (int l = lb; l < g->nlev; ++l) w += 6 * (size_t)g->lv[l].n_nodes;   // x, b
  return w;
}

size_t vbottom_lds_bytes(const tg_grid* g, int lb, size_t tsize) { return vb_words(g, lb) * tsize; }

// Algorithmic bytes of one bottom launch over the problems of list tv: per
// level the stored element matrices once per operator pass and the node-block
// inverses once per sweep, the coarsest inverse, and level lb's b and x in and
// result out.
double vbottom_bytes(const Batch* b, int tv) {
  const double ts = tv ? 8.0 : 4.0;
  const tg_mg_opts& mg = b->grids[0]->mg;
  double bytes = 0.0;
  for (int p : b->active) {
    const tg_grid* g = b->grids[p];
    const int lb = b->host_desc[p].vb_lb32 * (1 - tv) + b->host_desc[p].vb_lb64 * tv;
    if (lb >= g->nlev) continue;
    const int Lc = g->nlev - 1;
    for (int l = lb; l < Lc; ++l) {
      // level 1 reads its children's eight moduli, deeper levels their stored elements
      const double per_elem = l <= TG_MF_LEVELS ? 8.0 : (double)TG_GM_STRIDE;
      bytes += (mg.nu_pre + mg.nu_post) * per_elem * ts * g->lv[l].n_elem;
      bytes += (mg.nu_pre - 1 + mg.nu_post) * 9.0 * ts * g->lv[l].n_nodes;
      if (l + 1 < Lc) bytes += 9.0 * ts * g->lv[l + 1].n_nodes;
    }
    bytes += (double)g->ncoarse * g->ncoarse * ts;
    bytes += 3.0 * 3.0 * ts * g->lv[lb].n_nodes;
  }
  return bytes;
}

// First level from which the bottom kernel runs the cycle of g (TG_MAXLEV if
// none): the smallest lb >= 1 whose levels fit `lds` bytes with elements of
// `tsize` bytes and a direct coarsest solve.
int vbottom_level(const tg_grid* g, size_t tsize, size_t lds) {
  if (g->ncoarse <= 0 || g->nlev < 2) return TG_MAXLEV;
  for (int lb = 1; lb < g->nlev; ++lb)
    if (vb_words(g, lb) * tsize <= lds) return lb;
  return TG_MAXLEV;
}

template <class T> __device__ __forceinline__ const T* vb_cinv(const ProbDesc& P);
template <> __device__ __forceinline__ const double* vb_cinv<double>(const ProbDesc& P) { return P.Cinv64; }
template <> __device__ __forceinline__ const float* vb_cinv<float>(const ProbDesc& P) { return P.Cinv32; }

template <class T>
struct VbLev {
  int NX, NY, NZ, ex, ey, ez, nn, ne;
  T* x;
  T* b;
};

template <class T>
__device__ __forceinline__ VbLev<T> vb_lev(const LevelDesc& L, T* x, T* b) {
  return {L.NX, L.NY, L.NZ, L.ex, L.ey, L.ez, L.n_nodes, L.ex * L.ey * L.ez, x, b};
}

// eb[(3 a + c) * ne + e] = (K_e x_e)[3 a + c] for every element e of level l
// (level 1: the matrix-free moment form from the fine moduli; deeper levels:
// the stored mode-basis elements)
template <class T, bool L1>
__device__ __forceinline__ void vb_elements(const ProbDesc& P, int l, const LevelDesc& L, const VbLev<T>& V,
                                            T* eb) {
  const T TG_GLOBAL* Km = gp(fKm<T>(L));
  const int NXY = V.NX * V.NY;
  for (int e = threadIdx.x; e < V.ne; e += (int)blockDim.x) {
    const int i = e % V.ex, t = e / V.ex, j = t % V.ey, k = t / V.ey;
    const int n0 = i + V.NX * j + NXY * k;
    T ux[8], uy[8], uz[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int na = n0 + (a & 1) + V.NX * ((a >> 1) & 1) + NXY * (a >> 2);
      ux[a] = V.x[3 * na];
      uy[a] = V.x[3 * na + 1];
      uz[a] = V.x[3 * na + 2];
    }
    wht_fwd(ux);
    wht_fwd(uy);
    wht_fwd(uz);
    if (L1 && l <= TG_MF_LEVELS)
      elem_galerkin1<T>(ux, uy, uz, gp(fE<T>(P)), P.lv[0].ex, P.lv[0].ey, i, j, k,
                        (const T __attribute__((address_space(4)))*)G1V<T>(P));
    else
      elem_mode_stored<T, VbThreads<T, L1>::G>(ux, uy, uz, (const T*)Km, e);
    wht_inv(ux);
    wht_inv(uy);
    wht_inv(uz);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      eb[(3 * a + 0) * V.ne + e] = ux[a];
      eb[(3 * a + 1) * V.ne + e] = uy[a];
      eb[(3 * a + 2) * V.ne + e] = uz[a];
    }
  }
}

// (K x)_n from the element buffer: the elements around node (i, j, k) in the
// order dk, dj, di
template <class T>
__device__ __forceinline__ void vb_gather(const VbLev<T>& V, const T* eb, int i, int j, int k, T* kx) {
  kx[0] = kx[1] = kx[2] = T(0);
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di) {
        const int ei = i - 1 + di, ej = j - 1 + dj, ek = k - 1 + dk;
        if (ei < 0 || ei >= V.ex || ej < 0 || ej >= V.ey || ek < 0 || ek >= V.ez) continue;
        const int e = ei + V.ex * (ej + V.ey * ek);
        const int a = (1 - di) + 2 * (1 - dj) + 4 * (1 - dk);
#pragma unroll
        for (int c = 0; c < 3; ++c) kx[c] += eb[(3 * a + c) * V.ne + e];
      }
}

// One damped node-block Jacobi sweep x <- x + w D^-1 (b - K x) (RESID =
// false; after the element pass a node's update reads only its own x, so x
// is updated in place), or r = b - K x into rbuf (RESID = true); clamped
// nodes 0.
template <class T, bool RESID, bool L1>
__device__ void vb_sweep(const ProbDesc& P, int l, const VbLev<T>& V, T* eb, T* rbuf, T omega) {
  const LevelDesc& L = P.lv[l];
  vb_elements<T, L1>(P, l, L, V, eb);
  __syncthreads();
  for (int n = threadIdx.x; n < V.nn; n += (int)blockDim.x) {
    const int i = n % V.NX, t = n / V.NX, j = t % V.NY, k = t / V.NY;
    T* dst = RESID ? rbuf : V.x;
    if (i == 0) {
      if (RESID) dst[3 * n] = dst[3 * n + 1] = dst[3 * n + 2] = T(0);
      continue;
    }
    T kx[3];
    vb_gather<T>(V, eb, i, j, k, kx);
    const T r0 = V.b[3 * n] - kx[0], r1 = V.b[3 * n + 1] - kx[1], r2 = V.b[3 * n + 2] - kx[2];
    if (RESID) {
      dst[3 * n] = r0;
      dst[3 * n + 1] = r1;
      dst[3 * n + 2] = r2;
    } else {
      const T TG_GLOBAL* D = gp(fD<T>(L)) + 9LL * n;
      T xn[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        xn[c] = mad_(omega, mad_(D[3 * c + 2], r2, mad_(D[3 * c + 1], r1, D[3 * c] * r0)), V.x[3 * n + c]);
#pragma unroll
      for (int c = 0; c < 3; ++c) dst[3 * n + c] = xn[c];
    }
  }
  __syncthreads();
}

// b_c = P^T r (r = the fine residual in r[3 n + c]; full weighting, coarse
// x = 0 nodes clamped) and, if first_sweep, x_c = w D_c^-1 b_c
template <class T>
__device__ void vb_restrict(const VbLev<T>& F, const T* r, const LevelDesc& Lc, const VbLev<T>& C, T omega,
                            bool first_sweep) {
  for (int n = threadIdx.x; n < C.nn; n += (int)blockDim.x) {
    const int I = n % C.NX, t = n / C.NX, J = t % C.NY, K = t / C.NY;
    T s[3] = {T(0), T(0), T(0)};
    if (I > 0) {
      for (int dk = -1; dk <= 1; ++dk) {
        const int k = 2 * K + dk;
        if (k < 0 || k >= F.NZ) continue;
        for (int dj = -1; dj <= 1; ++dj) {
          const int j = 2 * J + dj;
          if (j < 0 || j >= F.NY) continue;
          for (int di = -1; di <= 1; ++di) {
            const int i = 2 * I + di;
            if (i < 0 || i >= F.NX) continue;
            const T w = T(1) / T(1 << ((di != 0) + (dj != 0) + (dk != 0)));
            const int f = i + F.NX * (j + F.NY * k);
#pragma unroll
            for (int c = 0; c < 3; ++c) s[c] = mad_(w, r[3 * f + c], s[c]);
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) C.b[3 * n + c] = s[c];
    if (first_sweep) {
      const T TG_GLOBAL* D = gp(fD<T>(Lc)) + 9LL * n;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        C.x[3 * n + c] = omega * mad_(D[3 * c + 2], s[2], mad_(D[3 * c + 1], s[1], D[3 * c] * s[0]));
    }
  }
  __syncthreads();
}

// x_f += P x_c (trilinear; clamped fine nodes untouched)
template <class T>
__device__ void vb_prolong(const VbLev<T>& F, const VbLev<T>& C) {
  for (int n = threadIdx.x; n < F.nn; n += (int)blockDim.x) {
    const int i = n % F.NX, t = n / F.NX, j = t % F.NY, k = t / F.NY;
    if (i == 0) continue;
    const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
    const T w = ((i & 1) ? T(0.5) : T(1)) * ((j & 1) ? T(0.5) : T(1)) * ((k & 1) ? T(0.5) : T(1));
    T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if ((c & 1) && !(i & 1)) continue;
      if ((c & 2) && !(j & 1)) continue;
      if ((c & 4) && !(k & 1)) continue;
      const int I = (c & 1) ? i1 : i0, J = (c & 2) ? j1 : j0, K = (c & 4) ? k1 : k0;
      const int m = I + C.NX * (J + C.NY * K);
      s0 = mad_(w, C.x[3 * m], s0);
      s1 = mad_(w, C.x[3 * m + 1], s1);
      s2 = mad_(w, C.x[3 * m + 2], s2);
    }
    F.x[3 * n] += s0;
    F.x[3 * n + 1] += s1;
    F.x[3 * n + 2] += s2;
  }
  __syncthreads();
}

// x = K_c^-1 b on the free DOFs of the coarsest level (free index
// 3 ((NX - 1) t + i - 1) + c of node i + NX t): eight lanes per row, each
// summing every eighth column, then a fixed butterfly over the eight
template <class T>
__device__ void vb_coarse(const ProbDesc& P, const VbLev<T>& C) {
  const int n = P.ncoarse;
  const T TG_GLOBAL* Ci = gp(vb_cinv<T>(P));
  const int part = threadIdx.x & 7, row0 = threadIdx.x >> 3;
  const int NXm = C.NX - 1;
  for (int q0 = 0; q0 < n; q0 += (int)blockDim.x / 8) {
    const int q = q0 + row0;
    T s = T(0);
    if (q < n)
#pragma unroll 8
      for (int c = part; c < n; c += 8) {
        const int fn = c / 3, node = fn % NXm + 1 + C.NX * (fn / NXm);
        s = mad_(Ci[(long long)q * n + c], C.b[3 * node + c % 3], s);
      }
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 4, 64);
    if (q < n && part == 0) {
      const int fn = q / 3, node = fn % NXm + 1 + C.NX * (fn / NXm);
      C.x[3 * node + q % 3] = s;
    }
  }
  __syncthreads();
}

// L1: some problem of the launch starts at level 1 (the moment-form
// operator is compiled in only then: it costs registers)
template <class T, bool L1>
__global__ __launch_bounds__((VbThreads<T, L1>::N)) void k_vbottom(const ProbDesc* __restrict__ probs,
                                                        const int2* __restrict__ work, int sfin, T omega,
                                                        int nu_pre, int nu_post) {
  extern __shared__ __align__(16) unsigned char vb_smem[];
  const int2 wi = work[blockIdx.x];
  const ProbDesc& P = probs[wi.x];
  TG_GATE(P);
  const int lb = sizeof(T) == 8 ? P.vb_lb64 : P.vb_lb32;
  const int Lc = P.nlev - 1;
  T* eb = (T*)vb_smem;
  T* rbuf = eb + 24 * (P.lv[lb].ex * P.lv[lb].ey * P.lv[lb].ez);
  // level l's x and b follow the element and residual buffers, level by level
  auto V = [&](int l) -> VbLev<T> {
    T* o = rbuf + 3 * P.lv[lb].n_nodes;
    for (int m = lb; m < l; ++m) o += 6 * P.lv[m].n_nodes;
    return vb_lev<T>(P.lv[l], o, o + 3 * P.lv[l].n_nodes);
  };
  // level-lb right-hand side and first sweep from the pools; deeper levels'
  // x start at zero (the coarsest keeps its clamped nodes at zero)
  {
    const LevelDesc& L = P.lv[lb];
    const T TG_GLOBAL* bg = gp(fpool<T>(L) + (long long)C_B * L.stride);
    const T TG_GLOBAL* xg = gp(fpool<T>(L) + (long long)C_XA * L.stride);
    const bool first = lb < Lc;
    const VbLev<T> Vb = V(lb);
    for (int q = threadIdx.x; q < 3 * Vb.nn; q += (int)blockDim.x) {
      Vb.b[q] = bg[q];
      Vb.x[q] = first ? xg[q] : T(0);
    }
    for (int l = lb + 1; l <= Lc; ++l) {
      const VbLev<T> Vl = V(l);
      for (int q = threadIdx.x; q < 3 * Vl.nn; q += (int)blockDim.x) Vl.x[q] = T(0);
    }
  }
  __syncthreads();
  // descend
  for (int l = lb; l < Lc; ++l) {
    const VbLev<T> Vl = V(l);
    for (int it = 1; it < nu_pre; ++it) vb_sweep<T, false, L1>(P, l, Vl, eb, rbuf, omega);
    vb_sweep<T, true, L1>(P, l, Vl, eb, rbuf, omega);
    vb_restrict<T>(Vl, rbuf, P.lv[l + 1], V(l + 1), omega, l + 1 < Lc);
  }
  vb_coarse<T>(P, V(Lc));
  // ascend
  for (int l = Lc - 1; l >= lb; --l) {
    const VbLev<T> Vl = V(l);
    vb_prolong<T>(Vl, V(l + 1));
    for (int it = 0; it < nu_post; ++it) vb_sweep<T, false, L1>(P, l, Vl, eb, rbuf, omega);
  }
  const LevelDesc& L = P.lv[lb];
  const VbLev<T> Vb = V(lb);
  T TG_GLOBAL* yg = gp(fpool<T>(L) + (long long)sfin * L.stride);
  for (int q = threadIdx.x; q < 3 * Vb.nn; q += (int)blockDim.x) yg[q] = Vb.x[q];
}

// Dynamic LDS the bottom kernel may take on the current device (the
// per-workgroup limit less a margin), with both kernels' limits raised to it
// once per device.
size_t vbottom_lds_limit() {
  static size_t lim[64] = {};
  static bool done[64] = {};
  static std::mutex mu;   // batches on several host threads
  std::lock_guard<std::mutex> lk(mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return 0;
  }
  if (!done[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
      (void)hipGetLastError();
      v = 0;
    }
    size_t l = v > 1024 ? (size_t)v - 1024 : 0;
    const void* kf[4] = {(const void*)k_vbottom<float, false>, (const void*)k_vbottom<float, true>,
                         (const void*)k_vbottom<double, false>, (const void*)k_vbottom<double, true>};
    bool ok = true;
    for (const void* k : kf)
      ok = ok && l && hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l) == hipSuccess;
    if (l && !ok) {
      (void)hipGetLastError();
      l = std::min<size_t>(l, 65536 - 1024);
    }
    lim[dev] = l;
    done[dev] = true;
  }
  return lim[dev];
}

template <class T>
int launch_vbottom(const Batch* b, const DevList& dl, size_t lds_bytes, int sfin, double omega, int nu_pre,
                   int nu_post, bool l1, hipStream_t s) {
  if (!dl.n) return TG_OK;
  if (l1)
    k_vbottom<T, true><<<dl.n, VbThreads<T, true>::N, lds_bytes, s>>>(b->desc_d, dl.ptr, sfin, T(omega), nu_pre, nu_post);
  else
    k_vbottom<T, false><<<dl.n, VbThreads<T, false>::N, lds_bytes, s>>>(b->desc_d, dl.ptr, sfin, T(omega), nu_pre, nu_post);
  return TG_OK;
}
template int launch_vbottom<float>(const Batch*, const DevList&, size_t, int, double, int, int, bool, hipStream_t);
template int launch_vbottom<double>(const Batch*, const DevList&, size_t, int, double, int, int, bool, hipStream_t);

}  // namespace tg
