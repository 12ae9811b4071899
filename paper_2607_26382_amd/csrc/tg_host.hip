// Host side of topoguard: element stiffness and transfer operators, grid
// setup, workspace sub-allocation, batch work lists.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "tg_internal.h"

namespace tg {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return TG_EHIP;
}

// ---------------------------------------------------------------------------
// Element stiffness of the unit cube (Sec. 3.1): trilinear hex8, isotropic,
// 2x2x2 Gauss on [0,1]^3.  Local node a = i + 2j + 4k, DOF 3a + c.  The
// integrand B^T D B is at most quadratic per coordinate, so the rule is exact.
// Assembled from the bilinear form lam div u div v + 2 mu eps(u):eps(v) via
// K[(a,i),(b,j)] = sum_g w_g [lam dNa_i dNb_j + mu dNa_j dNb_i + mu delta_ij gradNa.gradNb].
void build_ke(double E0, double nu, double* Ke) {
  const double lam = E0 * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = E0 / (2.0 * (1.0 + nu));
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  std::memset(Ke, 0, sizeof(double) * 576);
  for (int gz = 0; gz < 2; ++gz)
    for (int gy = 0; gy < 2; ++gy)
      for (int gx = 0; gx < 2; ++gx) {
        const double xyz[3] = {gp[gx], gp[gy], gp[gz]};
        const double w = 0.125;
        double dN[8][3];
        for (int a = 0; a < 8; ++a) {
          const int bit[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
          double f[3], df[3];
          for (int t = 0; t < 3; ++t) {
            f[t] = bit[t] ? xyz[t] : 1.0 - xyz[t];
            df[t] = bit[t] ? 1.0 : -1.0;
          }
          dN[a][0] = df[0] * f[1] * f[2];
          dN[a][1] = f[0] * df[1] * f[2];
          dN[a][2] = f[0] * f[1] * df[2];
        }
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b) {
            const double gg = dN[a][0] * dN[b][0] + dN[a][1] * dN[b][1] + dN[a][2] * dN[b][2];
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j) {
                double v = lam * dN[a][i] * dN[b][j] + mu * dN[a][j] * dN[b][i];
                if (i == j) v += mu * gg;
                Ke[(3 * a + i) * 24 + 3 * b + j] += w * v;
              }
          }
      }
  // exact symmetry (the rule is exact; remove the last-bit asymmetry)
  for (int r = 0; r < 24; ++r)
    for (int c = r + 1; c < 24; ++c) {
      const double v = 0.5 * (Ke[r * 24 + c] + Ke[c * 24 + r]);
      Ke[r * 24 + c] = Ke[c * 24 + r] = v;
    }
}

// P_c: interpolation from a coarse element's 24 DOFs to the 24 DOFs of its
// child c = (ci, cj, ck); fine local node a sits at fine offset (ci+ai, ...)
// in {0,1,2}^3 inside the coarse element, coarse corner b at (2bi, 2bj, 2bk).
// 1D trilinear weight: 1 - |pos - 2b| / 2.
void build_child_prolong(double* Pc) {
  std::memset(Pc, 0, sizeof(double) * 8 * 576);
  for (int c = 0; c < 8; ++c) {
    const int co[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    for (int a = 0; a < 8; ++a) {
      const int ab[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
      for (int b = 0; b < 8; ++b) {
        const int bb[3] = {b & 1, (b >> 1) & 1, (b >> 2) & 1};
        double w = 1.0;
        for (int t = 0; t < 3; ++t) {
          const int pos = co[t] + ab[t];
          w *= 1.0 - std::abs(pos - 2 * bb[t]) / 2.0;
        }
        for (int comp = 0; comp < 3; ++comp) Pc[c * 576 + (3 * a + comp) * 24 + 3 * b + comp] = w;
      }
    }
  }
}

void build_child_galerkin(const double* Ke, const double* Pc, double* G) {
  for (int c = 0; c < 8; ++c) {
    const double* P = Pc + c * 576;
    double T[576];
    for (int r = 0; r < 24; ++r)
      for (int s = 0; s < 24; ++s) {
        double t = 0.0;
        for (int a = 0; a < 24; ++a) t += Ke[r * 24 + a] * P[a * 24 + s];
        T[r * 24 + s] = t;
      }
    for (int r = 0; r < 24; ++r)
      for (int s = 0; s < 24; ++s) {
        double t = 0.0;
        for (int a = 0; a < 24; ++a) t += P[a * 24 + r] * T[a * 24 + s];
        G[c * 576 + r * 24 + s] = t;
      }
  }
}

// ---------------------------------------------------------------------------
// bump allocator over a caller workspace
struct Bump {
  char* base;
  size_t off = 0, cap;
  bool dry;
  Bump(void* b, size_t c, bool d) : base((char*)b), cap(c), dry(d) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = dry ? nullptr : (T*)(base + off);
    off += count * sizeof(T);
    return p;
  }
};

// Slot stride: a whole number of reduction chunks, so the Krylov sweeps can
// read every chunk in full (the tail stays zero: the workspace is cleared at
// bind and those sweeps write zeros there).
static long long stride_of(long long n_dof) { return (n_dof + TG_VCHUNK - 1) / TG_VCHUNK * TG_VCHUNK; }

static size_t list_capacity(const std::vector<tg_grid*>& gs) {
  size_t c = 64;
  for (auto* g : gs) {
    for (int l = 0; l < g->nlev; ++l) {
      const size_t tiles = (g->lv[l].n_nodes + TG_NODE_TILE - 1) / TG_NODE_TILE;
      c += 2 * tiles + 1;
      c += (l == 0) ? (g->lv[0].n_elem + 255) / 256 : g->lv[l].n_elem;
    }
    c += g->lv[0].n_chunks + 1;
    c += 2;   // the V-cycle bottom lists
    for (int l = 0; l < g->nlev; ++l) c += zm_tiles(g, l, 1);
    for (int l = 0; l + 1 < g->nlev; ++l) c += rz_tiles(g, l, 1);
    c += zm_tiles(g, 0, 1);
  }
  return c;
}

static void batch_layout(Bump& bp, Batch* b, int n, size_t lcap) {
  b->desc_d = bp.take<ProbDesc>(n);
  b->list_d = bp.take<int2>(lcap);
  b->sc_d = bp.take<double>(n + 8);
  b->flag_d = bp.take<int>(n + 64);
  b->feat_d = bp.take<double>(8 * (size_t)n);
  b->list_cap = lcap;
}

static void grid_layout(tg_grid* g, Bump& bp, int mmax) {
  ProbDesc& D = g->desc;
  std::memset(&D, 0, sizeof(D));
  D.nlev = g->nlev;
  D.ncoarse = g->ncoarse;
  D.Ke64 = bp.take<double>(576);
  D.Ke32 = bp.take<float>(576);
  D.G64 = bp.take<double>(8 * 576);
  D.Pc64 = bp.take<double>(8 * 576);
  D.G1v64 = bp.take<double>(TG_G1_NVAL);
  D.G1v32 = bp.take<float>(TG_G1_NVAL);
  D.E64 = bp.take<double>(g->lv[0].n_elem);
  D.E32 = bp.take<float>(g->lv[0].n_elem);
  D.cc = bp.take<int>(2 * (size_t)g->lv[0].n_elem);
  for (int l = 0; l < g->nlev; ++l) {
    LevelDesc& L = D.lv[l];
    const LevelHost& H = g->lv[l];
    L.ex = H.ex;
    L.ey = H.ey;
    L.ez = H.ez;
    L.NX = H.ex + 1;
    L.NY = H.ey + 1;
    L.NZ = H.ez + 1;
    L.n_nodes = (int)H.n_nodes;
    L.n_chunks = H.n_chunks;
    L.stride = H.stride;
    const int ns64 = (l == 0) ? n_slots0(mmax) : C_NSLOTS;
    L.vec64 = bp.take<double>((size_t)ns64 * H.stride);
    L.vec32 = bp.take<float>((size_t)C_NSLOTS * H.stride);
    if (l >= 1) {
      L.Kel64 = bp.take<double>((size_t)H.n_elem * 576);
    }
    if (l > TG_MF_LEVELS) {
      L.Km64 = bp.take<double>((size_t)gm_elems(H.n_elem) * TG_GM_STRIDE);
      L.Km32 = bp.take<float>((size_t)gm_elems(H.n_elem) * TG_GM_STRIDE);
    }
    L.Dinv64 = bp.take<double>((size_t)9 * H.n_nodes);
    L.Dinv32 = bp.take<float>((size_t)9 * H.n_nodes);
  }
  const size_t nc = g->ncoarse;
  D.Cinv64 = bp.take<double>(nc * nc);
  D.Cinv32 = bp.take<float>(nc * nc);
  D.Cwork = bp.take<double>(2 * nc * nc);
  g->sl.init(mmax, TG_HIST_CAP);
  D.small = bp.take<double>(g->sl.total);
  D.part = bp.take<double>((size_t)TG_PART_W * g->lv[0].n_chunks);
}

size_t batch_ws_bytes_for(const std::vector<tg_grid*>& gs) {
  Bump bp(nullptr, 0, true);
  Batch tmp;
  batch_layout(bp, &tmp, (int)gs.size(), list_capacity(gs));
  return bp.off + 256;
}

static void drop_graphs(Batch* b) {
  for (auto& kv : b->graphs) hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

Batch::~Batch() {
  drop_graphs(this);
  if (cap_stream) hipStreamDestroy(cap_stream);
}

int batch_init(Batch* b, int n, tg_grid* const* grids) {
  if (n <= 0) return fail(TG_EINVAL, "batch needs at least one grid");
  b->grids.assign(grids, grids + n);
  b->n = n;
  for (auto* g : b->grids) {
    if (!g || !g->bound) return fail(TG_ESTATE, "every grid of a batch needs a bound workspace");
    if (g->mmax != b->grids[0]->mmax)
      return fail(TG_EINVAL, "grids of one batch must be bound with the same max_restart");
    if (std::memcmp(g->Ke, b->grids[0]->Ke, sizeof(g->Ke)) != 0)
      return fail(TG_EINVAL, "grids of one batch must share E0 and nu (one element stiffness)");
    if (g->mg.omega != b->grids[0]->mg.omega || g->mg.nu_pre != b->grids[0]->mg.nu_pre ||
        g->mg.nu_post != b->grids[0]->mg.nu_post)
      return fail(TG_EINVAL, "grids of one batch must share the smoother options");
  }
  b->sc_h.assign(n + 8, 0.0);
  b->host_desc.resize(n);
  batch_choose_zc(b);
  return TG_OK;
}

int batch_bind(Batch* b, void* ws, size_t bytes) {
  const size_t need = batch_ws_bytes_for(b->grids);
  if (!ws || bytes < need) return fail(TG_EWORKSPACE, "batch workspace too small");
  Bump bp(ws, bytes, false);
  b->lists_valid = false;
  drop_graphs(b);
  batch_layout(bp, b, b->n, list_capacity(b->grids));
  b->ws = ws;
  b->ws_bytes = bytes;
  return TG_OK;
}

// The height a launch uses: the chosen one, capped while only a few problems
// run (zc_cap, see batch_set_active).
int batch_zc_run(const Batch* b, int p, int l) { return std::min(batch_zc(b, p, l), b->zc_cap[l]); }

int batch_zc(const Batch* b, int p, int l) {
  const tg_grid* g = b->grids[p];
  if (!b->zc_size.empty()) {
    const auto it = b->zc_size.find({g->nx, g->ny, g->nz});
    if (it != b->zc_size.end() && it->second[l] > 0) return it->second[l];
  }
  return b->zc[l];
}

unsigned long long batch_zc_hash(const Batch* b) {
  unsigned long long h = 1469598103934665603ull;
  auto mix = [&](long long v) {
    for (int q = 0; q < 8; ++q) {
      h ^= (unsigned long long)((v >> (8 * q)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  for (int l = 0; l < TG_MAXLEV; ++l) mix(b->zc[l]);
  for (int l = 0; l < TG_MAXLEV; ++l) mix(b->zc_cap[l]);
  for (const auto& kv : b->zc_size) {
    for (int d : kv.first) mix(d);
    for (int z : kv.second) mix(z);
  }
  return h;
}

int batch_upload_desc(Batch* b, hipStream_t s) {
  for (int p = 0; p < b->n; ++p) {
    b->host_desc[p] = b->grids[p]->desc;
    b->host_desc[p].gate = b->gated ? b->sc_d + p : nullptr;
    const size_t lim = vbottom_lds_limit();
    b->host_desc[p].vb_lb32 = vbottom_level(b->grids[p], sizeof(float), lim);
    b->host_desc[p].vb_lb64 = vbottom_level(b->grids[p], sizeof(double), lim);
    for (int l = 0; l < b->grids[p]->nlev; ++l)
      b->host_desc[p].lv[l].zc = zm_height(b->grids[p]->lv[l].ez + 1, batch_zc_run(b, p, l));
  }
  TG_HIP(hipMemcpyAsync(b->desc_d, b->host_desc.data(), sizeof(ProbDesc) * b->n, hipMemcpyHostToDevice, s));
  return TG_OK;
}

// z-tile caps for a subset of the batch: while few problems run (the tail of a
// ladder), a level whose z-march launch would have fewer than 1024
// workgroups at the chosen heights gets the tallest height in {16, 12, 8, 6,
// 4, 3} that restores 1024, else 2.  Shorter tiles redo one element layer
// more often but shorten each workgroup's serial march, and the device is
// mostly idle then.  Results do not depend on the heights.
static void batch_tile_caps(const Batch* b, const std::vector<int>& active, int* cap) {
  for (int l = 0; l < TG_MAXLEV; ++l) cap[l] = 1 << 30;
  if ((int)active.size() >= b->n) return;
  for (int l = 0; l < TG_MAXLEV; ++l) {
    auto tiles = [&](int c) {
      long long t = 0;
      for (int p : active) {
        const tg_grid* g = b->grids[p];
        if (l < g->nlev - 1) t += zm_tiles(g, l, std::min(batch_zc(b, p, l), c));
      }
      return t;
    };
    const long long t0 = tiles(1 << 30);
    if (t0 == 0 || t0 >= 1024) continue;
    int pick = 2;
    for (int c : {16, 12, 8, 6, 4, 3})
      if (tiles(c) >= 1024) {
        pick = c;
        break;
      }
    cap[l] = pick;
  }
}

int batch_set_active(Batch* b, const std::vector<int>& active, hipStream_t s, bool with_elem) {
  {
    int cap[TG_MAXLEV];
    batch_tile_caps(b, active, cap);
    if (!std::equal(cap, cap + TG_MAXLEV, b->zc_cap)) {
      // the descriptors carry the tile heights the kernels use
      std::copy(cap, cap + TG_MAXLEV, b->zc_cap);
      const int rc = batch_upload_desc(b, s);
      if (rc) return rc;
    }
  }
  const unsigned long long zh = batch_zc_hash(b);
  if (b->lists_valid && b->lists_active == active && (b->lists_elem || !with_elem) && b->lists_zc_hash == zh) {
    b->active = active;
    return TG_OK;   // the lists on the device already describe this set
  }
  b->lists_valid = false;
  // the previous host list buffer may still be in flight: synchronize first
  TG_HIP(hipStreamSynchronize(s));
  b->active = active;
  std::vector<int2>& H = b->host_lists;
  H.clear();
  std::vector<std::pair<size_t, size_t>> rng;   // (offset, count) per list
  auto begin = [&]() { return H.size(); };
  b->maxlev = 0;
  for (int p : active) b->maxlev = std::max(b->maxlev, b->grids[p]->nlev);
  size_t o;
  auto finish = [&](DevList& d, size_t start) {
    d.n = (int)(H.size() - start);
    d.ptr = b->list_d + start;
  };
  for (int l = 0; l < TG_MAXLEV; ++l) {
    o = begin();
    for (int p : active) {
      tg_grid* g = b->grids[p];
      if (l >= g->nlev) continue;
      const int tiles = (int)((g->lv[l].n_nodes + TG_NODE_TILE - 1) / TG_NODE_TILE);
      for (int t = 0; t < tiles; ++t) H.push_back(make_int2(p, t));
    }
    finish(b->node[l], o);
    o = begin();
    for (int p : active) {
      tg_grid* g = b->grids[p];
      if (l >= g->nlev - 1) continue;
      const int tiles = (int)((g->lv[l].n_nodes + TG_NODE_TILE - 1) / TG_NODE_TILE);
      for (int t = 0; t < tiles; ++t) H.push_back(make_int2(p, t));
    }
    finish(b->smooth[l], o);
    o = begin();
    for (int p : active)
      if (l == b->grids[p]->nlev - 1) H.push_back(make_int2(p, 0));
    finish(b->coarse[l], o);
    o = begin();
    if (with_elem) {
      for (int p : active) {
        tg_grid* g = b->grids[p];
        if (l >= g->nlev) continue;
        const long long cnt = (l == 0) ? (g->lv[0].n_elem + 255) / 256 : g->lv[l].n_elem;
        for (long long t = 0; t < cnt; ++t) H.push_back(make_int2(p, (int)t));
      }
    }
    finish(b->elem[l], o);
  }
  o = begin();
  for (int p : active)
    for (int c = 0; c < b->grids[p]->lv[0].n_chunks; ++c) H.push_back(make_int2(p, c));
  finish(b->vec, o);
  o = begin();
  for (int p : active) H.push_back(make_int2(p, 0));
  finish(b->prob, o);
  o = begin();
  for (int p : active)
    for (int t = 0, nt = zm_tiles(b->grids[p], 0, batch_zc_run(b, p, 0)); t < nt; ++t) H.push_back(make_int2(p, t));
  finish(b->fine, o);
  for (int l = 0; l < TG_MAXLEV; ++l) {
    o = begin();
    for (int p : active)
      if (l < b->grids[p]->nlev - 1)
        for (int t = 0, nt = zm_tiles(b->grids[p], l, batch_zc_run(b, p, l)); t < nt; ++t) H.push_back(make_int2(p, t));
    finish(b->zm_s[l], o);
    o = begin();
    for (int p : active)
      if (l < b->grids[p]->nlev - 1)
        for (int t = 0, nt = rz_tiles(b->grids[p], l, batch_zc_run(b, p, l)); t < nt; ++t) H.push_back(make_int2(p, t));
    finish(b->zm_r[l], o);
  }
  // the one-launch V-cycle bottom (per vector type): its problems, its LDS,
  // and the levels that still need level-by-level launches
  {
    const size_t lim = vbottom_lds_limit();
    for (int t = 0; t < 2; ++t) {
      const size_t ts = t ? sizeof(double) : sizeof(float);
      o = begin();
      size_t lds = 0;
      bool l1 = false;
      for (int l = 0; l < TG_MAXLEV; ++l) b->vb_need[t][l] = false;
      for (int p : active) {
        const tg_grid* g = b->grids[p];
        const int lb = vbottom_level(g, ts, lim);
        for (int l = 0; l < std::min(lb, g->nlev); ++l) b->vb_need[t][l] = true;
        if (lb < g->nlev) {
          H.push_back(make_int2(p, 0));
          lds = std::max(lds, vbottom_lds_bytes(g, lb, ts));
          l1 = l1 || lb <= TG_MF_LEVELS;
        }
      }
      finish(b->vb[t], o);
      b->vb_lds[t] = lds;
      b->vb_l1[t] = l1;
    }
  }
  if (H.size() > b->list_cap) return fail(TG_EWORKSPACE, "work-list capacity exceeded");
  if (!H.empty())
    TG_HIP(hipMemcpyAsync(b->list_d, H.data(), H.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  b->lists_valid = true;
  b->lists_elem = with_elem;
  b->lists_active = active;
  b->lists_zc_hash = zh;
  // the list layout is a function of (active set, zc, elem flag): equal
  // signatures mean identical device lists at identical addresses
  unsigned long long h = 1469598103934665603ull;
  auto mix = [&](long long v) {
    for (int q = 0; q < 8; ++q) {
      h ^= (unsigned long long)((v >> (8 * q)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix((long long)active.size());
  for (int p : active) mix(p);
  mix((long long)zh);
  mix(with_elem ? 1 : 0);
  b->lists_sig = h;
  return TG_OK;
}

int batch_read_status(Batch* b, hipStream_t s) {
  TG_HIP(hipMemcpyAsync(b->sc_h.data(), b->sc_d, sizeof(double) * b->n, hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  return TG_OK;
}

// ---------------------------------------------------------------------------
// grid setup
static int free_dof(int x, int y, int z) { return 3 * x * (y + 1) * (z + 1); }

int grid_setup(int nx, int ny, int nz, double E0, double nu, const tg_mg_opts* mg, tg_grid** out) {
  if (!out) return fail(TG_EINVAL, "out is NULL");
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1) return fail(TG_EINVAL, "grid dimensions must be >= 1");
  const long long nodes = (long long)(nx + 1) * (ny + 1) * (nz + 1);
  if (nodes * 3 > (1LL << 31) - 1) return fail(TG_EINVAL, "grid too large (DOF index exceeds int32)");
  if (!(E0 > 0) || !(nu > -1.0 && nu < 0.5)) return fail(TG_EINVAL, "need E0 > 0 and -1 < nu < 0.5");
  tg_mg_opts o;
  tg_default_mg_opts(&o);
  if (mg) o = *mg;
  if (o.max_levels < 0 || o.max_levels > TG_MAXLEV) return fail(TG_EINVAL, "max_levels out of range");
  if (o.max_coarse_dof < 3 || o.max_coarse_dof > TG_MAX_COARSE)
    return fail(TG_EINVAL, "max_coarse_dof must be in [3, 512]");
  if (!(o.omega > 0 && o.omega < 2) || o.nu_pre < 1 || o.nu_post < 1 || o.nu_pre > 16 || o.nu_post > 16)
    return fail(TG_EINVAL, "smoother options out of range (0<omega<2, 1<=nu<=16)");
  tg_grid* g = new tg_grid();
  g->nx = nx;
  g->ny = ny;
  g->nz = nz;
  g->E0 = E0;
  g->nu = nu;
  g->mg = o;
  int dims[TG_MAXLEV][3];
  int L = 1;
  dims[0][0] = nx;
  dims[0][1] = ny;
  dims[0][2] = nz;
  const int maxl = o.max_levels ? o.max_levels : TG_MAXLEV;
  while (L < maxl) {
    const int x = dims[L - 1][0], y = dims[L - 1][1], z = dims[L - 1][2];
    if (free_dof(x, y, z) <= o.max_coarse_dof) break;
    if ((x | y | z) & 1) break;
    if (x / 2 < 2 || y / 2 < 2 || z / 2 < 2) break;
    dims[L][0] = x / 2;
    dims[L][1] = y / 2;
    dims[L][2] = z / 2;
    ++L;
  }
  const int cfree = free_dof(dims[L - 1][0], dims[L - 1][1], dims[L - 1][2]);
  // A coarsest level above TG_MAX_COARSE free DOFs has no dense direct solve:
  // the operator and the guard still work, the V-cycle is refused.
  g->coarse_ok = cfree <= TG_MAX_COARSE;
  g->nlev = L;
  for (int l = 0; l < L; ++l) {
    LevelHost& H = g->lv[l];
    H.ex = dims[l][0];
    H.ey = dims[l][1];
    H.ez = dims[l][2];
    H.n_elem = (long long)H.ex * H.ey * H.ez;
    H.n_nodes = (long long)(H.ex + 1) * (H.ey + 1) * (H.ez + 1);
    H.n_dof = 3 * H.n_nodes;
    H.stride = stride_of(H.n_dof);
    H.n_chunks = (int)((H.n_dof + TG_VCHUNK - 1) / TG_VCHUNK);
    H.zc = 16;
  }
  g->ncoarse = g->coarse_ok ? cfree : 0;
  g->ncoarse_true = cfree;
  build_ke(E0, nu, g->Ke);
  {
    int rc = mode_coef_from_ke(g->Ke, &g->mc64, &g->mc32);
    if (!rc) rc = galerkin1_values(g->Ke, g->g1v);
    if (rc) {
      delete g;
      return rc;
    }
  }
  build_child_prolong(g->Pc);
  build_child_galerkin(g->Ke, g->Pc, g->G);
  *out = g;
  return TG_OK;
}

size_t grid_ws_bytes(const tg_grid* g, int mmax) {
  Bump bp(nullptr, 0, true);
  tg_grid tmp = *g;
  grid_layout(&tmp, bp, mmax);
  std::vector<tg_grid*> one{&tmp};
  bp.take<char>(batch_ws_bytes_for(one));
  return bp.off + 256;
}

int grid_bind(tg_grid* g, void* ws, size_t bytes, int mmax) {
  if (mmax < 1 || mmax > TG_MAX_RESTART) return fail(TG_EINVAL, "max_restart must be in [1, 126]");
  const size_t need = grid_ws_bytes(g, mmax);
  if (!ws || bytes < need)
    return fail(TG_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  if (((uintptr_t)ws) & 255) return fail(TG_EINVAL, "workspace must be 256-byte aligned");
  Bump bp(ws, bytes, false);
  grid_layout(g, bp, mmax);
  TG_HIP(hipMemset(ws, 0, bp.off));   // vector padding must read as zero
  g->mmax = mmax;
  g->ws = ws;
  g->ws_bytes = bytes;
  g->bound = true;
  g->density_set = false;
  // constant tables
  float ke32[576];
  for (int q = 0; q < 576; ++q) ke32[q] = (float)g->Ke[q];
  TG_HIP(hipMemcpy((void*)g->desc.Ke64, g->Ke, sizeof(g->Ke), hipMemcpyHostToDevice));
  TG_HIP(hipMemcpy((void*)g->desc.Ke32, ke32, sizeof(ke32), hipMemcpyHostToDevice));
  TG_HIP(hipMemcpy((void*)g->desc.G64, g->G, sizeof(g->G), hipMemcpyHostToDevice));
  TG_HIP(hipMemcpy((void*)g->desc.Pc64, g->Pc, sizeof(g->Pc), hipMemcpyHostToDevice));
  float g1v32[TG_G1_NVAL];
  for (int q = 0; q < TG_G1_NVAL; ++q) g1v32[q] = (float)g->g1v[q];
  TG_HIP(hipMemcpy((void*)g->desc.G1v64, g->g1v, sizeof(g->g1v), hipMemcpyHostToDevice));
  TG_HIP(hipMemcpy((void*)g->desc.G1v32, g1v32, sizeof(g1v32), hipMemcpyHostToDevice));
  // batch of one inside the same workspace
  delete g->self;
  g->self = new Batch();
  tg_grid* self = g;
  int rc = batch_init(g->self, 1, &self);
  if (rc) return rc;
  const size_t bb = batch_ws_bytes_for(g->self->grids);
  char* bws = bp.take<char>(bb);
  return batch_bind(g->self, bws, bb);
}

}  // namespace tg

// ===========================================================================
// C ABI: errors, defaults, grid
using namespace tg;

extern "C" {

const char* tg_last_error(void) { return tg::g_err.c_str(); }

void tg_default_mg_opts(tg_mg_opts* o) {
  if (!o) return;
  o->max_levels = 0;
  o->max_coarse_dof = 300;
  o->omega = 0.6;
  o->nu_pre = 2;
  o->nu_post = 2;
}

void tg_default_solver_opts(tg_solver_opts* o) {
  if (!o) return;
  o->restart = 30;
  o->max_iters = 200;
  o->tol = 1e-6;
  o->prec = TG_F64;
  o->cgs_passes = 2;
  o->graphs = 0;
  o->breakdown = 1e-14;
  o->sync_every = 8;
}

int tg_setup_grid(int nx, int ny, int nz, double E0, double nu, const tg_mg_opts* mg, tg_grid** out) {
  return grid_setup(nx, ny, nz, E0, nu, mg, out);
}

void tg_destroy(tg_grid* g) {
  if (!g) return;
  delete g->self;
  delete g;
}

int tg_get_grid_info(const tg_grid* g, tg_grid_info* info) {
  if (!g || !info) return fail(TG_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->nx = g->nx;
  info->ny = g->ny;
  info->nz = g->nz;
  info->n_elem = g->lv[0].n_elem;
  info->n_nodes = g->lv[0].n_nodes;
  info->n_dof = g->lv[0].n_dof;
  info->n_free = 3LL * g->nx * (g->ny + 1) * (g->nz + 1);
  info->n_levels = g->nlev;
  for (int l = 0; l < g->nlev; ++l) {
    info->level_dims[l][0] = g->lv[l].ex;
    info->level_dims[l][1] = g->lv[l].ey;
    info->level_dims[l][2] = g->lv[l].ez;
  }
  info->coarse_free_dof = g->ncoarse_true;
  return TG_OK;
}

int tg_get_ke(const tg_grid* g, double* ke_h) {
  if (!g || !ke_h) return fail(TG_EINVAL, "NULL argument");
  std::memcpy(ke_h, g->Ke, sizeof(g->Ke));
  return TG_OK;
}

int tg_edge_load(const tg_grid* g, double* f_h) {
  if (!g || !f_h) return fail(TG_EINVAL, "NULL argument");
  const long long NX = g->nx + 1, NY = g->ny + 1;
  std::memset(f_h, 0, sizeof(double) * g->lv[0].n_dof);
  for (int j = 0; j <= g->ny; ++j) {
    double w = 1.0 / g->ny;
    if (j == 0 || j == g->ny) w *= 0.5;
    const long long n = g->nx + NX * j;   // k = 0
    f_h[3 * n + 2] -= w;
  }
  (void)NY;
  return TG_OK;
}

int tg_workspace_bytes(const tg_grid* g, int max_restart, size_t* bytes) {
  if (!g || !bytes) return fail(TG_EINVAL, "NULL argument");
  if (max_restart < 1 || max_restart > TG_MAX_RESTART) return fail(TG_EINVAL, "max_restart must be in [1, 126]");
  *bytes = grid_ws_bytes(g, max_restart);
  return TG_OK;
}

int tg_bind_workspace(tg_grid* g, void* ws_d, size_t bytes, int max_restart) {
  if (!g) return fail(TG_EINVAL, "NULL grid");
  return grid_bind(g, ws_d, bytes, max_restart);
}

}  // extern "C"
