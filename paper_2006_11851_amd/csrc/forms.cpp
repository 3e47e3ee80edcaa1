// Accelerated search forms: placeholders until their kernels land.
#include "bf16_learned.hpp"

namespace pts {

void search_brute_bf16(Ctx*, ExView, const Index&, const float*, int, int, const pts_estep_params&, const float*,
                       int64_t, int32_t*) {
  fail(PTS_ERR_UNSUPPORTED, "BRUTE_BF16 not available");
}

int64_t search_learned(Ctx*, ExView, const Index&, const float*, int, int, const pts_estep_params&, const float*,
                       int64_t, int32_t*, bool, bool) {
  fail(PTS_ERR_UNSUPPORTED, "learned modes not available");
}

}  // namespace pts

extern "C" {
int pts_mlp_init(pts_ctx*, int, int, int, uint64_t) { return PTS_ERR_UNSUPPORTED; }
int pts_mlp_n_params(pts_ctx*, int64_t*) { return PTS_ERR_UNSUPPORTED; }
int pts_mlp_get_weights(pts_ctx*, float*) { return PTS_ERR_UNSUPPORTED; }
int pts_mlp_set_weights(pts_ctx*, const float*) { return PTS_ERR_UNSUPPORTED; }
int pts_mlp_set_input_scale(pts_ctx*, const float*) { return PTS_ERR_UNSUPPORTED; }
int pts_mlp_forward(pts_ctx*, const float*, int64_t, int, float*) { return PTS_ERR_UNSUPPORTED; }
int pts_mlp_loss_grad(pts_ctx*, const float*, const int32_t*, int64_t, int, float*, float*) { return PTS_ERR_UNSUPPORTED; }
int pts_mlp_train(pts_ctx*, const float*, const int32_t*, int64_t, const pts_train_params*, float*) { return PTS_ERR_UNSUPPORTED; }
int pts_mlp_propose(pts_ctx*, const float*, int64_t, int, int32_t*, float*) { return PTS_ERR_UNSUPPORTED; }
}
