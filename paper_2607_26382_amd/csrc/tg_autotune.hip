// Autotuner for the z-march kernels: per level, time the V-cycle smoothing
// sweep of the actual batch for each candidate z-tile height and keep the
// fastest; in a batch of several grid sizes, then choose each size's height
// in turn (the other sizes fixed), again timing the sweep over the whole
// batch.  Results are cached per batch signature (grid dimensions of every
// problem and the working precision) for the life of the process, and
// optionally in a text file named by TG_AUTOTUNE_CACHE (one line per
// signature: the key, the count of values, the level-wide heights, then the
// heights of each size in order of first appearance).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <sstream>

#include "tg_internal.h"

namespace tg {

namespace {
std::mutex g_mu;
std::map<std::string, std::vector<int>> g_cache;
bool g_loaded = false;

void load_file() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("TG_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[4096];
  while (std::fscanf(f, "%4095s", key) == 1) {
    int cnt = 0;
    if (std::fscanf(f, "%d", &cnt) != 1 || cnt < TG_MAXLEV || cnt > 64 * TG_MAXLEV) break;
    std::vector<int> v(cnt);
    for (int q = 0; q < cnt; ++q)
      if (std::fscanf(f, "%d", &v[q]) != 1) v[q] = 0;
    g_cache[key] = v;
  }
  std::fclose(f);
}

void save_file() {
  const char* path = std::getenv("TG_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  for (auto& kv : g_cache) {
    std::fprintf(f, "%s %d", kv.first.c_str(), (int)kv.second.size());
    for (int x : kv.second) std::fprintf(f, " %d", x);
    std::fprintf(f, "\n");
  }
  std::fclose(f);
}
}  // namespace

std::string batch_signature(const Batch* b, int prec) {
  std::ostringstream o;
  o << "p" << prec << "_n" << b->n;
  // problems in order of appearance, run-length encoded by grid size
  int i = 0;
  while (i < b->n) {
    int j = i;
    const tg_grid* g = b->grids[i];
    while (j < b->n && b->grids[j]->nx == g->nx && b->grids[j]->ny == g->ny && b->grids[j]->nz == g->nz) ++j;
    o << "_" << (j - i) << "x" << g->nx << "." << g->ny << "." << g->nz;
    i = j;
  }
  return o.str();
}

// Grid sizes of the batch in order of first appearance.
static std::vector<std::array<int, 3>> batch_sizes(const Batch* b) {
  std::vector<std::array<int, 3>> v;
  for (auto* g : b->grids) {
    const std::array<int, 3> d = {g->nx, g->ny, g->nz};
    if (std::find(v.begin(), v.end(), d) == v.end()) v.push_back(d);
  }
  return v;
}

// Applies cached tile heights if this batch has been tuned before.
bool autotune_lookup(Batch* b, int prec) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file();
  auto it = g_cache.find(batch_signature(b, prec));
  if (it == g_cache.end()) return false;
  const std::vector<int>& v = it->second;
  for (int l = 0; l < TG_MAXLEV; ++l)
    if (v[l] > 0) b->zc[l] = v[l];
  b->zc_size.clear();
  const auto sizes = batch_sizes(b);
  if (sizes.size() > 1 && v.size() == (sizes.size() + 1) * TG_MAXLEV)
    for (size_t q = 0; q < sizes.size(); ++q)
      for (int l = 0; l < TG_MAXLEV; ++l) b->zc_size[sizes[q]][l] = v[(q + 1) * TG_MAXLEV + l];
  return true;
}

int autotune_batch(Batch* b, int prec, hipStream_t s, double* best_us, bool force) {
  if (prec < TG_F64 || prec > TG_BF16X3MFMA) return fail(TG_EINVAL, "unknown precision");
  for (int l = 0; l < TG_MAXLEV && best_us; ++l) best_us[l] = -1.0;
  if (!force && autotune_lookup(b, prec)) return batch_upload_desc(b, s);
  std::vector<int> all(b->n);
  for (int i = 0; i < b->n; ++i) {
    all[i] = i;
    if (!b->grids[i]->density_set) return fail(TG_ESTATE, "autotune needs set_density first");
  }
  hipEvent_t e0, e1;
  TG_HIP(hipEventCreate(&e0));
  TG_HIP(hipEventCreate(&e1));
  int rc = TG_OK;
  b->zc_size.clear();
  const int mf = prec == TG_BF16MFMA ? 1 : prec == TG_BF16X3MFMA ? 2 : 0;
  // time of the level-l smoothing sweep over the whole batch with the
  // current heights (microseconds, mean of 3 after one untimed sweep)
  auto timed = [&](int l, double& us) -> int {
    int r;
    if ((r = batch_upload_desc(b, s)) || (r = batch_set_active(b, all, s))) return r;
    auto sweep = [&]() {
      // damped Jacobi sweep on the level's scratch vectors (values irrelevant)
      if (prec == TG_F64)
        return launch_fine<double>(b, b->zm_s[l], l, 2, l == 0 ? S_VXA : C_XA, nullptr,
                                   l == 0 ? S_VB : C_B, nullptr, l == 0 ? S_VXB : C_XB, nullptr, 0.6, s);
      if (l == 0 && mf)
        return launch_fine_mfma(b, b->zm_s[0], 2, mf == 2, C_XA, nullptr, C_B, nullptr, C_XB, nullptr, 0.6,
                                false, s);
      return launch_fine<float>(b, b->zm_s[l], l, 2, C_XA, nullptr, C_B, nullptr, C_XB, nullptr, 0.6, s);
    };
    if ((r = sweep())) return r;
    TG_HIP(hipEventRecord(e0, s));
    const int reps = 3;
    for (int q = 0; q < reps; ++q)
      if ((r = sweep())) return r;
    TG_HIP(hipEventRecord(e1, s));
    TG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    TG_HIP(hipEventElapsedTime(&ms, e0, e1));
    us = 1e3 * ms / reps;
    return TG_OK;
  };
  for (int l = 0; l < TG_MAXLEV && rc == TG_OK; ++l) {
    bool any = false;
    for (auto* g : b->grids) any = any || (l < g->nlev - 1);
    if (!any) continue;
    // candidate heights: the balanced heights ceil(NZ / t) of every grid at
    // this level (t z-tiles, so the tile count can match the number of
    // resident workgroups) plus a few small ones
    std::vector<int> cand = {2, 3, 4, 6, 8};
    for (auto* g : b->grids) {
      if (l >= g->nlev - 1) continue;
      const int NZ = g->lv[l].ez + 1;
      for (int t = 1; t <= std::min(NZ, 64); ++t) cand.push_back((NZ + t - 1) / t);
    }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    double best = 1e30;
    int pick = b->zc[l];
    for (int c : cand) {
      b->zc[l] = c;
      double us = 0.0;
      if ((rc = timed(l, us))) break;
      if (us < best) {
        best = us;
        pick = c;
      }
    }
    b->zc[l] = pick;
    if (best_us) best_us[l] = best;
  }
  // several grid sizes: each size's height in turn, the others fixed
  const auto sizes = batch_sizes(b);
  if (rc == TG_OK && sizes.size() > 1) {
    for (const auto& d : sizes) b->zc_size[d].fill(0);
    for (int l = 0; l < TG_MAXLEV && rc == TG_OK; ++l) {
      for (const auto& d : sizes) {
        const tg_grid* g = nullptr;
        for (auto* gg : b->grids)
          if (gg->nx == d[0] && gg->ny == d[1] && gg->nz == d[2]) g = gg;
        if (l >= g->nlev - 1) continue;
        const int NZ = g->lv[l].ez + 1;
        std::vector<int> cand = {2, 3, 4, 6, 8, b->zc[l]};
        for (int t = 1; t <= std::min(NZ, 64); ++t) cand.push_back((NZ + t - 1) / t);
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        double best = 1e30;
        int pick = b->zc[l];
        for (int c : cand) {
          b->zc_size[d][l] = c;
          double us = 0.0;
          if ((rc = timed(l, us))) break;
          if (us < best) {
            best = us;
            pick = c;
          }
        }
        b->zc_size[d][l] = pick;
        if (rc) break;
        if (best_us && best < best_us[l]) best_us[l] = best;
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if ((rc = batch_upload_desc(b, s))) return rc;
  std::vector<int> v(b->zc, b->zc + TG_MAXLEV);
  if (sizes.size() > 1)
    for (const auto& d : sizes) v.insert(v.end(), b->zc_size[d].begin(), b->zc_size[d].end());
  std::lock_guard<std::mutex> lk(g_mu);
  load_file();
  g_cache[batch_signature(b, prec)] = v;
  save_file();
  return TG_OK;
}

}  // namespace tg
