// Learned first-floor selector (placeholder until the kernels land).
#include "tg_internal.h"

struct tg_mlp {
  int dummy;
};

namespace tg {
int mlp_select(const tg_mlp*, const std::vector<std::array<float, 8>>&, std::vector<int>&, hipStream_t) {
  return fail(TG_EINVAL, "MLP selector not available in this build");
}
int density_features(Batch*, const std::vector<int>&, const double* const*, double, double,
                     std::vector<std::array<float, 8>>&, hipStream_t) {
  return fail(TG_EINVAL, "density features not available in this build");
}
}  // namespace tg

extern "C" {
int tg_mlp_workspace_bytes(int, size_t*) { return tg::fail(TG_EINVAL, "MLP not available in this build"); }
int tg_mlp_create(void*, size_t, int, tg_mlp**) { return tg::fail(TG_EINVAL, "MLP not available in this build"); }
void tg_mlp_destroy(tg_mlp*) {}
int tg_mlp_set_params(tg_mlp*, const float*, const float*, const float*, void*) {
  return tg::fail(TG_EINVAL, "MLP not available in this build");
}
int tg_mlp_get_params(const tg_mlp*, float*, void*) { return tg::fail(TG_EINVAL, "MLP not available in this build"); }
int tg_mlp_forward(const tg_mlp*, const float*, int, float*, void*) {
  return tg::fail(TG_EINVAL, "MLP not available in this build");
}
int tg_mlp_train_step(tg_mlp*, const float*, const int*, int, float, float*, float*, void*) {
  return tg::fail(TG_EINVAL, "MLP not available in this build");
}
}
