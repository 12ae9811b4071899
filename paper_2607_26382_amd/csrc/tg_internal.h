// Internal layout of the topoguard library (gfx950).
//
// Every solver kernel is batch-aware: a launch covers a work list of
// (problem, tile) pairs, one pair per workgroup, and each problem carries a
// device descriptor with its grid dimensions and its device arrays.  A single
// solve is a batch of one; uneven batches reuse the same kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/topoguard.h"
#include "tg_galerkin1_pattern.h"

#define TG_MAXLEV 8
#define TG_NODE_TILE 256     // nodes per workgroup for node-centred kernels
#define TG_VCHUNK 2048       // DOFs per workgroup for vector kernels
#define TG_VBLOCK 256        // threads per vector workgroup
#define TG_PART_W 256        // max partial sums of one sweep (2 max_restart + 3)
#define TG_MAX_RESTART 126
#define TG_MAX_COARSE 512    // max free DOFs of the coarsest level
#define TG_HIST_CAP 4096     // residual-history capacity per problem
#define TG_GM_STRIDE 152    // stored entries per mode-basis element matrix (TG_GM_NU = 150, padded)
// The stored mode-basis element matrices of a level are laid out in blocks of
// 64 elements: entry v of element e belongs to 16-byte piece v / W (W = 16 /
// sizeof entry), and piece p of element e sits at piece index
// ((e / 64) * (TG_GM_STRIDE / W) + p) * 64 + e % 64.  The 64 lanes of a wave
// reading piece p of 64 consecutive elements thus read 1 KB of consecutive
// memory.  Arrays hold ceil(n_elem / 64) * 64 elements.
__host__ __device__ inline long long gm_index(long long e, int v, int W) {
  const long long np = TG_GM_STRIDE / W;
  return ((((e >> 6) * np + v / W) << 6) + (e & 63)) * W + v % W;
}
__host__ __device__ inline long long gm_elems(long long n_elem) { return (n_elem + 63) & ~63LL; }
#define TG_MF_LEVELS 1       // levels 1..TG_MF_LEVELS apply the Galerkin operator matrix-free

namespace tg {

// Device pointers taken from descriptors have no known address space, so the
// compiler emits flat memory instructions for them (which also count against
// the LDS wait counter).  gp() re-tags a pointer as global memory.
#define TG_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const T TG_GLOBAL* gp(const T* p) {
  return (const T TG_GLOBAL*)p;
}
template <class T>
__device__ __forceinline__ T TG_GLOBAL* gp(T* p) {
  return (T TG_GLOBAL*)p;
}

// Workgroups are dealt to the 8 XCDs round robin (workgroup i runs on XCD
// i mod 8) and each XCD has its own L2.  Giving every XCD a contiguous range
// of the work list keeps neighbouring tiles, which share halo nodes and
// partly used cache lines, in one L2.  A bijection on [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
#define TG_HIP(call)                                        \
  do {                                                      \
    hipError_t _e = (call);                                 \
    if (_e != hipSuccess) return ::tg::hip_fail(_e, #call); \
  } while (0)

// ---------------------------------------------------------------------------
// Per-level device view.  Vectors at a level live in two slot pools (FP64 and
// FP32); slot s of a problem sits at pool + s * stride.
struct LevelDesc {
  int ex, ey, ez;           // elements
  int NX, NY, NZ;           // nodes per dimension (= elements + 1)
  int n_nodes;
  int n_chunks;             // ceil(3 n_nodes / TG_VCHUNK)
  int zc;                   // z-tile height (node layers) of the z-march kernels
  int pad_;
  long long stride;         // slot stride in elements (>= 3 n_nodes, 64-aligned)
  double* vec64;
  float* vec32;
  double* Kel64;            // levels >= 1: 576 values per element (row-major 24x24)
  double* Km64;             // levels > TG_MF_LEVELS: the element matrix in the mode
  float* Km32;              // basis, TG_GM_NU values padded to TG_GM_STRIDE per element
  double* Dinv64;           // 9 values per node (3x3 inverse of the node block)
  float* Dinv32;
};

struct ProbDesc {
  int nlev;
  int ncoarse;              // free DOFs at the coarsest level
  double rho_min;
  double* E64;              // fine element moduli
  float* E32;
  double* Cinv64;           // coarsest dense inverse, ncoarse x ncoarse (row-major)
  float* Cinv32;
  double* Cwork;            // coarsest assembly / factorization scratch
  const double* Ke64;       // shared element stiffness (576)
  const float* Ke32;
  const double* G64;        // 8 x 576: child Galerkin matrices P_c^T Ke P_c
  const double* Pc64;       // 8 x 576: child prolongations P_c (fine 24 x coarse 24)
  const double* G1v64;      // TG_G1_NVAL values of the level-1 moment matrices
  const float* G1v32;
  double* small;            // per-problem FGMRES scalars (SmallLayout)
  double* part;             // reduction partials: TG_PART_W x n_chunks(level 0)
  const double* ext0;       // per-call external vectors (batched copy in/out)
  double* ext1;
  int* cc;                  // 2 x n_elem: component labels, clamped-face flags
  // Inside FGMRES: this problem's entry of the status gather.  The kernels
  // of an Arnoldi step return at once (whole workgroups) when it is no
  // longer TG_RUNNING, so several steps run between host reads of the
  // status.  Null elsewhere.
  const double* gate;
  // first level of the V-cycle run by the one-launch bottom kernel for FP32
  // and FP64 vectors (TG_MAXLEV: none)
  int vb_lb32, vb_lb64;
  LevelDesc lv[TG_MAXLEV];
};
// Workgroup-uniform early exit of a step kernel for a problem that stopped.
#define TG_GATE(P)                                       \
  do {                                                   \
    if ((P).gate && *(P).gate != TG_RUNNING) return;     \
  } while (0)

// Level-0 FP64 slots.
enum { S_F = 0, S_X = 1, S_R = 2, S_W = 3, S_T = 4, S_VB = 5, S_VXA = 6, S_VXB = 7, S_VR = 8, S_V0 = 9 };
inline int slot_V(int j) { return S_V0 + j; }
inline int slot_Z(int mmax, int j) { return S_V0 + mmax + 1 + j; }
inline int n_slots0(int mmax) { return S_V0 + 2 * mmax + 1; }
// V-cycle slots at levels >= 1 (both pools) and in the level-0 FP32 pool.
enum { C_B = 0, C_XA = 1, C_XB = 2, C_R = 3, C_NSLOTS = 4 };

// Per-problem small FGMRES state (doubles).
struct SmallLayout {
  int mmax, cap;
  int H, g, cs, sn, y, h, tmp, scal, hist, total;
  void init(int m, int c) {
    mmax = m;
    cap = c;
    int o = 0;
    H = o;   o += (m + 1) * m;   // column-major: H[i + (m+1) j]
    g = o;   o += m + 1;
    cs = o;  o += m;
    sn = o;  o += m;
    y = o;   o += m;
    h = o;   o += TG_PART_W;     // accumulated projection coefficients
    tmp = o; o += TG_PART_W;     // multi-dot result of the current pass
    scal = o; o += 32;
    hist = o; o += c + 1;
    total = (o + 31) & ~31;
  }
};
// scalar slots inside small + scal
enum { SC_BNORM = 0, SC_BETA = 1, SC_HN = 2, SC_STATUS = 3, SC_ITERS = 4, SC_JDONE = 5,
       SC_EST = 6, SC_TRUE = 7, SC_INV = 8, SC_FLAG = 9, SC_RHO = 10, SC_GJ = 11 };
#define TG_RUNNING (-1.0)

// Ke of a cube in the per-component polynomial-mode basis has 8 distinct
// coefficients (values divided by 64, the squared norm of a mode vector).
template <class T>
struct ModeCoef {
  T d, o, s, p, q, r, t, w;
};

struct LevelHost {
  int ex, ey, ez;
  long long n_elem, n_nodes, n_dof, stride;
  int n_chunks;
  int zc;                   // z-tile height of the z-march kernels
};

struct Batch;

}  // namespace tg

struct tg_grid {
  int nx = 0, ny = 0, nz = 0;
  double E0 = 1, nu = 0.3;
  tg_mg_opts mg;
  int nlev = 0;
  tg::LevelHost lv[TG_MAXLEV];
  int ncoarse = 0;            // free DOFs of the coarsest level (0 if no direct solve)
  int ncoarse_true = 0;
  bool coarse_ok = true;
  double Ke[576];
  tg::ModeCoef<double> mc64;
  tg::ModeCoef<float> mc32;
  double G[8 * 576];
  double Pc[8 * 576];
  double g1v[TG_G1_NVAL];  // level-1 moment-matrix values (pattern kG1Pattern)
  // workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int mmax = 0;
  int cap = 0;
  tg::SmallLayout sl;
  tg::ProbDesc desc;          // host copy of this grid's device descriptor
  bool bound = false;
  bool density_set = false;
  bool numeric_bad = false;   // coarsest factorization met a non-positive pivot
  double p = 0, rho_min = 0;
  tg::Batch* self = nullptr;  // batch of one for single-grid calls
};

namespace tg {

struct DevList {
  const int2* ptr = nullptr;
  int n = 0;
};

struct Batch {
  std::vector<tg_grid*> grids;
  int n = 0;
  int maxlev = 0;
  ProbDesc* desc_d = nullptr;     // device descriptors (n)
  int2* list_d = nullptr;         // device work-list storage
  size_t list_cap = 0;            // capacity in int2
  double* sc_d = nullptr;         // device status gather (n doubles)
  int* flag_d = nullptr;          // per-problem validation flags (set_density)
  double* feat_d = nullptr;       // per-problem density statistics (8 each)
  double p = 3.0;                 // SIMP exponent of the current set_density
  std::vector<double> sc_h;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<int> active;
  DevList node[TG_MAXLEV], smooth[TG_MAXLEV], coarse[TG_MAXLEV], elem[TG_MAXLEV], vec, prob;
  DevList fine;                   // level-0 z-march tiles, all problems
  DevList zm_s[TG_MAXLEV];        // level-l z-march tiles, problems where l is not the coarsest
  DevList zm_r[TG_MAXLEV];        // level-l residual-restriction tiles (same problems)
  // one-launch V-cycle bottom, per vector type (0: FP32, 1: FP64): the problems
  // it serves, its dynamic LDS, and per level whether any problem still needs
  // the level-by-level launches there
  DevList vb[2];
  size_t vb_lds[2] = {0, 0};
  bool vb_l1[2] = {false, false};   // some problem's bottom starts at level 1
  bool vb_need[2][TG_MAXLEV] = {};
  std::vector<int2> host_lists;   // kept alive until the next synchronization
  std::vector<ProbDesc> host_desc;
  int zc[TG_MAXLEV] = {};         // z-tile height per level for this batch
  // caps on the heights while only part of the batch runs (batch_set_active)
  int zc_cap[TG_MAXLEV] = {1 << 30, 1 << 30, 1 << 30, 1 << 30, 1 << 30, 1 << 30, 1 << 30, 1 << 30};
  // z-tile heights per grid size (nx, ny, nz) and level where the autotuner
  // chose one for that size (0: zc[l])
  std::map<std::array<int, 3>, std::array<int, TG_MAXLEV>> zc_size;
  bool gated = false;             // descriptors carry the step gate (FGMRES)
  // key of the work lists currently on the device (rebuilt only when it changes)
  bool lists_valid = false;
  bool lists_elem = false;
  std::vector<int> lists_active;
  unsigned long long lists_zc_hash = 0;
  unsigned long long lists_sig = 0;     // hash of what the device lists encode (set, zc, elem)
  // captured FGMRES steps (graph replay), keyed by lists epoch and step shape
  hipStream_t cap_stream = nullptr;
  std::map<std::string, hipGraphExec_t> graphs;
  ~Batch();
};

size_t batch_ws_bytes_for(const std::vector<tg_grid*>& grids);
int batch_init(Batch* b, int n, tg_grid* const* grids);
int batch_bind(Batch* b, void* ws, size_t bytes);
int batch_upload_desc(Batch* b, hipStream_t s);
int batch_set_active(Batch* b, const std::vector<int>& active, hipStream_t s, bool with_elem = false);
int batch_read_status(Batch* b, hipStream_t s);   // fills sc_h from small[SC_STATUS]
int batch_zc(const Batch* b, int p, int l);       // z-tile height of problem p at level l
int batch_zc_run(const Batch* b, int p, int l);   // the same, capped for a small running set
unsigned long long batch_zc_hash(const Batch* b); // of zc and every per-size choice

// launch wrappers (tg_kernels.hip)
int k_set_density(Batch* b, hipStream_t s);
int k_apply(Batch* b, int prec, int sx, const void* ex, int sy, void* ey, hipStream_t s);
int k_residual64(Batch* b, int sb, int sx, int sy, hipStream_t s);
int k_dots2(Batch* b, int sbase, int nv, int sq, int sw, hipStream_t s);
int k_update2(Batch* b, int sbase, int nv, int sq, int sw, int snext, int cap, double tol, double brk,
              hipStream_t s);
int k_vcycle(Batch* b, int prec, int in_is_f32, int sb, const void* eb, int out_is_f32, int sy,
             void* ey, hipStream_t s, int in_scale_sc = -1);   // input scaled by small[scal + in_scale_sc]
int k_copy_ext(Batch* b, int dir, int slot, hipStream_t s);  // dir 0: ext0 -> slot; 1: slot -> ext1
int k_fill0(Batch* b, int slot, double v, hipStream_t s);
int k_copy0(Batch* b, int src, int dst, hipStream_t s);
int k_multidot(Batch* b, int sbase, int nv, int sw, int with_self, hipStream_t s);
int k_reduce(Batch* b, int nv, int mode, int dst, int save_k, hipStream_t s);  // 0: h=tmp 1: h+=tmp 2: tmp
int k_update(Batch* b, int sbase, int nv, int sw, int coef_is_tmp, hipStream_t s);
// fused sweep: w -= V coef, then partial dots of the updated w with V (ndot
// vectors) and, if with_self, with itself (chunk-local, deterministic).
int k_update_dots(Batch* b, int sbase, int nv, int sw, int coef_is_tmp, int ndot, int with_self,
                  hipStream_t s);
int k_scale_to(Batch* b, int src, int dst, int sc_index, hipStream_t s);
int k_cycle_start(Batch* b, int k, int cap, double tol, hipStream_t s);
int k_arnoldi(Batch* b, int j, int k, int cap, double tol, double brk, hipStream_t s);
int k_lsq_update(Batch* b, int mmax, int jmax, hipStream_t s);
// small[SC_TRUE] from R and F dots; to_status: also into the status gather
int k_true_eta(Batch* b, hipStream_t s, bool to_status = true);
int k_init_small(Batch* b, hipStream_t s);
// level primitives of host-stepped cycles (FP64; x, bb, y external vectors
// of level l): op 0 y = K x, 1 y = bb - K x, 2 y = x + omega D^-1 (bb - K x);
// the fused residual-restriction into pool slot slot_next of level l + 1;
// xf += P ec; y = K_c^-1 bb at the coarsest level
enum { LV_APPLY = 0, LV_RESID = 1, LV_SMOOTH = 2 };
int level_op64(Batch* b, int l, int op, const double* x, const double* bb, double* y, double omega, hipStream_t s);
int level_restrict64(Batch* b, int l, const double* x, const double* bb, int slot_next, hipStream_t s);
int level_prolong64(Batch* b, int l, const double* ec, double* xf, hipStream_t s);
int level_coarse64(Batch* b, int l, const double* bb, double* y, hipStream_t s);

// policy pieces shared by the fixed-cycle and the adaptive-stack policies
// (tg_solver.hip, tg_mlp.hip): probe features from a history, Eq. trigger,
// the network's first rung, the six density statistics
void probe_feats(const double* hist, int kstop, double* r50, double* r100);
int rule_fires(const tg_policy* pol, double r50, double r100);
int mlp_select(const tg_mlp* m, const std::vector<std::array<float, 8>>& feats, std::vector<int>& k0,
               hipStream_t s);
int density_features(Batch* b, const std::vector<int>& which, const double* const* rho_d, double p,
                     double rho0, std::vector<std::array<float, 8>>& out, hipStream_t s);

// kernel-class timer (tg_timer.hip)
bool timer_on();
void timer_suspend(bool on);
void* timer_begin(int kind, hipStream_t s);
void timer_end(void* h, double bytes, hipStream_t s);
void timer_harvest();

// fine-level z-march kernels (tg_fine.hip)
int mode_coef_from_ke(const double* Ke, ModeCoef<double>* out64, ModeCoef<float>* out32);
int galerkin1_values(const double* Ke, double* out);
int zm_height(int NZ, int zmax);
int zm_tiles(const tg_grid* g, int l, int zmax);
int rz_tiles(const tg_grid* g, int l, int zmax);
void batch_choose_zc(Batch* b);
template <class T>
// op 3 (residual fused with the restriction): sy is the next level's
// right-hand-side slot; sy2 >= 0 also writes that level's first Jacobi sweep
// from zero into slot sy2
int launch_fine(const Batch* b, const DevList& dl, int l, int op, int sx, const void* ex, int sb,
                const void* eb, int sy, void* ey, double omega, hipStream_t s, int sy2 = -1, int vbskip = 0);
// the bottom of the V-cycle in one launch per problem (levels vb_lb.. in LDS)
int vbottom_level(const tg_grid* g, size_t tsize, size_t lds);
size_t vbottom_lds_limit();
size_t vbottom_lds_bytes(const tg_grid* g, int lb, size_t tsize);
double vbottom_bytes(const Batch* b, int tv);
template <class T>
int launch_vbottom(const Batch* b, const DevList& dl, size_t lds_bytes, int sfin, double omega, int nu_pre,
                   int nu_post, bool l1, hipStream_t s);
int launch_fine_smooth_out64(const Batch* b, const DevList& dl, int sx, int sb, int sy, double omega,
                             hipStream_t s);
int launch_fine_mfma(const Batch* b, const DevList& dl, int op, bool split, int sx, const void* ex, int sb,
                     const void* eb, int sy, void* ey, double omega, bool out64, hipStream_t s,
                     int sy2 = -1);

// autotuner (tg_autotune.hip)
std::string batch_signature(const Batch* b, int prec);
bool autotune_lookup(Batch* b, int prec);
int autotune_batch(Batch* b, int prec, hipStream_t s, double* best_us, bool force);

// host helpers (tg_host.cpp)
void build_ke(double E0, double nu, double* Ke);
void build_child_prolong(double* Pc);           // 8 x 24 x 24
void build_child_galerkin(const double* Ke, const double* Pc, double* G);
}  // namespace tg
